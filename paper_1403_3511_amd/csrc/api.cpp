// C ABI entry points: argument validation, device-block uploads and dispatch.
#include <cmath>
#include <cstring>
#include <string>

#include "hs_internal.h"

namespace hs {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
int32_t fail(int32_t code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
int32_t hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return HS_E_HIP;
}

int32_t launch_copy_coeffs(const hs_pot_s *p, void *pot_dev, const double *coef, hipStream_t s);
int32_t launch_step(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, void *pot_dev,
                    int32_t dtype, double t, double *t_dev, double h, int m, int reorth, void *c,
                    void *ws, double *diag, hipStream_t s);
int64_t step_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype, int m);
int64_t m4_apply_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype);
int64_t step4_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype, int m);
int32_t launch_apply_m4(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, const void *pot1,
                        const void *pot2, int32_t dtype, double h, const void *x, void *y, void *ws,
                        hipStream_t s);
int32_t launch_step_m4(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, void *pot1,
                       void *pot2, int32_t dtype, double t, double *t_dev, double h, int m, int reorth,
                       void *c, void *ws, double *diag, hipStream_t s);

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace hs

extern "C" int32_t hs_last_error(char *buf, size_t len) {
  if (!buf || len == 0) return HS_E_INVALID;
  const std::string &e = hs::g_last_error;
  const size_t n = std::min(len - 1, e.size());
  std::memcpy(buf, e.data(), n);
  buf[n] = 0;
  return HS_OK;
}

extern "C" const char *hs_version(void) { return "1.0 gfx950"; }

extern "C" int32_t hs_pot_upload(hs_pot pot, void *dev, int64_t bytes, void *stream) {
  if (!pot || !dev) return hs::fail(HS_E_INVALID, "hs_pot_upload: NULL argument");
  if (bytes < pot->dev_bytes) return hs::fail(HS_E_WORKSPACE, "hs_pot_upload: device buffer too small");
  if (!hs::aligned16(dev)) return hs::fail(HS_E_INVALID, "hs_pot_upload: device pointer not 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // host image of the static part (base, amp, freq, phase, M); pinned so the copy is
  // asynchronous; kept alive by the handle until it is destroyed or re-uploaded
  static_assert(sizeof(double) == 8, "");
  std::vector<uint8_t> img(pot->dev_bytes, 0);
  auto put = [&](int64_t off, const double *src, int64_t n) {
    if (n > 0) std::memcpy(img.data() + off, src, n * 8);
  };
  put(pot->off_base, pot->base.data(), pot->nterms);
  put(pot->off_amp, pot->amp.data(), pot->nterms);
  put(pot->off_freq, pot->freq.data(), pot->nterms);
  put(pot->off_phase, pot->phase.data(), pot->nterms);
  if (pot->fused) put(pot->off_M, pot->M.data(), (int64_t)pot->nslots * pot->nterms);
  if (!pot->cptr.empty()) {  // combination table of a split program: cptr | cidx | cterm
    int32_t *ct = reinterpret_cast<int32_t *>(img.data() + pot->off_comb);
    std::memcpy(ct, pot->cptr.data(), 4 * pot->cptr.size());
    std::memcpy(ct + pot->cptr.size(), pot->cidx.data(), 4 * pot->cidx.size());
    std::memcpy(ct + pot->cptr.size() + pot->cidx.size(), pot->cterm.data(), 4 * pot->cterm.size());
  }
  void *pinned = nullptr;
  HS_HIP(hipHostMalloc(&pinned, pot->dev_bytes, hipHostMallocDefault));
  std::memcpy(pinned, img.data(), pot->dev_bytes);
  hipError_t e = hipMemcpyAsync(dev, pinned, pot->dev_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    (void)hipHostFree(pinned);
    return hs::hip_fail(e, "hs_pot_upload: hipMemcpyAsync");
  }
  // the staging buffer must outlive the copy: wait for it here (upload is not hot)
  e = hipStreamSynchronize(s);
  (void)hipHostFree(pinned);
  if (e != hipSuccess) return hs::hip_fail(e, "hs_pot_upload: hipStreamSynchronize");
  return hs::launch_set_time(pot, dev, 0.0, nullptr, 0.0, s);
}

extern "C" int32_t hs_pot_set_time(hs_pot pot, void *pot_dev, double t, const double *t_dev,
                                   void *stream) {
  if (!pot || !pot_dev) return hs::fail(HS_E_INVALID, "hs_pot_set_time: NULL argument");
  if (!t_dev && !std::isfinite(t)) return hs::fail(HS_E_NONFINITE, "hs_pot_set_time: t not finite");
  return hs::launch_set_time(pot, pot_dev, t, t_dev, 0.0, static_cast<hipStream_t>(stream));
}

extern "C" int32_t hs_pot_set_form(hs_pot pot, int32_t form) {
  if (!pot) return hs::fail(HS_E_INVALID, "hs_pot_set_form: NULL handle");
  if (form != HS_FORM_PAPER && form != HS_FORM_SYM) return hs::fail(HS_E_INVALID, "hs_pot_set_form: unknown form");
  if (form == HS_FORM_SYM && !pot->fused)
    return hs::fail(HS_E_UNSUPPORTED, "hs_pot_set_form: the symmetrised form needs a potential of the fused class");
  pot->form = form;
  return HS_OK;
}

extern "C" int32_t hs_pot_set_coeffs_device(hs_pot pot, void *pot_dev, const double *coef_dev,
                                            void *stream) {
  if (!pot || !pot_dev || !coef_dev) return hs::fail(HS_E_INVALID, "hs_pot_set_coeffs_device: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  pot->x2 = pot->x2_struct;  // values now come from the device
  int32_t st = hs::launch_copy_coeffs(pot, pot_dev, coef_dev, s);
  if (st != HS_OK) return st;
  return hs::launch_set_time(pot, pot_dev, 0.0, nullptr, 0.0, s);
}

extern "C" int32_t hs_workspace_bytes(hs_index idx, hs_pot pot, int32_t dtype, int32_t m,
                                      int64_t *bytes) {
  if (!idx || !pot || !bytes) return hs::fail(HS_E_INVALID, "hs_workspace_bytes: NULL argument");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_workspace_bytes: bad dtype");
  if (m < 0 || m > 32) return hs::fail(HS_E_INVALID, "hs_workspace_bytes: m out of range 0..32");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_workspace_bytes: potential and index differ in N");
  *bytes = hs::step_workspace_bytes(idx, pot, dtype, m);
  return HS_OK;
}

extern "C" int32_t hs_apply_h(hs_index idx, const void *idx_dev, hs_pot pot, const void *pot_dev,
                              int32_t dtype, const void *c, void *y, void *ws, void *stream) {
  if (!idx || !pot || !idx_dev || !pot_dev || !c || !y)
    return hs::fail(HS_E_INVALID, "hs_apply_h: NULL argument");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_apply_h: potential and index differ in N");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_apply_h: bad dtype");
  if (c == y) return hs::fail(HS_E_INVALID, "hs_apply_h: input and output must differ");
  if (!hs::aligned16(c) || !hs::aligned16(y) || !hs::aligned16(idx_dev) || !hs::aligned16(pot_dev))
    return hs::fail(HS_E_INVALID, "hs_apply_h: device pointer not 16-byte aligned");
  if (hs::apply_workspace_bytes(idx, pot, dtype) > 0 && (!ws || !hs::aligned16(ws)))
    return hs::fail(HS_E_WORKSPACE, "hs_apply_h: this potential needs a workspace");
  return hs::launch_apply(idx, idx_dev, pot, pot_dev, dtype, c, y, ws,
                          static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr, nullptr);
}

extern "C" int32_t hs_apply_x(hs_index idx, const void *idx_dev, int32_t axis, int32_t dtype, const void *c,
                              void *y, void *stream) {
  if (!idx || !idx_dev || !c || !y) return hs::fail(HS_E_INVALID, "hs_apply_x: NULL argument");
  if (axis < 0 || axis >= idx->N) return hs::fail(HS_E_INVALID, "hs_apply_x: axis out of range 0..N-1");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_apply_x: bad dtype");
  if (c == y) return hs::fail(HS_E_INVALID, "hs_apply_x: input and output must differ");
  if (!hs::aligned16(c) || !hs::aligned16(y) || !hs::aligned16(idx_dev))
    return hs::fail(HS_E_INVALID, "hs_apply_x: device pointer not 16-byte aligned");
  return hs::launch_apply_x(idx, idx_dev, axis, dtype, c, y, static_cast<hipStream_t>(stream));
}

extern "C" int32_t hs_step(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev,
                           int32_t dtype, double t, double *t_dev, double h, int32_t m,
                           int32_t reorth, void *c, void *ws, double *diag_dev, void *stream) {
  if (!idx || !pot || !idx_dev || !pot_dev || !c || !ws)
    return hs::fail(HS_E_INVALID, "hs_step: NULL argument");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_step: potential and index differ in N");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_step: bad dtype");
  if (m < 1 || m > 32) return hs::fail(HS_E_INVALID, "hs_step: m out of range 1..32");
  if (!std::isfinite(h) || (!t_dev && !std::isfinite(t))) return hs::fail(HS_E_NONFINITE, "hs_step: t or h not finite");
  if (!hs::aligned16(c) || !hs::aligned16(ws) || !hs::aligned16(idx_dev) || !hs::aligned16(pot_dev))
    return hs::fail(HS_E_INVALID, "hs_step: device pointer not 16-byte aligned");
  return hs::launch_step(idx, idx_dev, pot, pot_dev, dtype, t, t_dev, h, m, reorth, c, ws, diag_dev,
                         static_cast<hipStream_t>(stream));
}

extern "C" int32_t hs_debug_checks(int32_t *built) {
  if (!built) return hs::fail(HS_E_INVALID, "hs_debug_checks: built is NULL");
#ifdef HS_DEBUG_BOUNDS
  *built = 1;
#else
  *built = 0;
#endif
  return HS_OK;
}

extern "C" int32_t hs_index_debug_read(hs_index idx, const void *idx_dev, uint32_t *counts_host, int32_t clear,
                                       void *stream) {
  if (!idx || !idx_dev || !counts_host) return hs::fail(HS_E_INVALID, "hs_index_debug_read: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t *dbg = const_cast<uint8_t *>(static_cast<const uint8_t *>(idx_dev)) + idx->off_dbg;
  uint32_t words[2] = {0, 0};
  HS_HIP(hipMemcpyAsync(words, dbg, sizeof(words), hipMemcpyDeviceToHost, s));
  HS_HIP(hipStreamSynchronize(s));
  counts_host[0] = words[0];
  counts_host[1] = words[1];
  if (clear) {
    const uint32_t zero[2] = {0, 0};
    HS_HIP(hipMemcpyAsync(dbg, zero, sizeof(zero), hipMemcpyHostToDevice, s));
    HS_HIP(hipStreamSynchronize(s));
  }
  return HS_OK;
}

extern "C" int32_t hs_set_small_step_rows(int64_t rows) {
  if (rows < 0) return hs::fail(HS_E_INVALID, "hs_set_small_step_rows: negative row count");
  hs::set_small_step_rows(rows);
  return HS_OK;
}

extern "C" int32_t hs_get_small_step_rows(int64_t *rows) {
  if (!rows) return hs::fail(HS_E_INVALID, "hs_get_small_step_rows: rows is NULL");
  *rows = hs::small_step_rows();
  return HS_OK;
}

extern "C" int32_t hs_propagate(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev, int32_t dtype,
                                double t0, double *t_dev, double h, int32_t m, int32_t reorth, int64_t nsteps,
                                void *c, void *ws, void *stream) {
  if (!idx || !pot || !idx_dev || !pot_dev || !c || !ws)
    return hs::fail(HS_E_INVALID, "hs_propagate: NULL argument");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_propagate: potential and index differ in N");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_propagate: bad dtype");
  if (m < 1 || m > 32) return hs::fail(HS_E_INVALID, "hs_propagate: m out of range 1..32");
  if (nsteps < 0) return hs::fail(HS_E_INVALID, "hs_propagate: negative step count");
  if (!std::isfinite(h) || (!t_dev && !std::isfinite(t0)))
    return hs::fail(HS_E_NONFINITE, "hs_propagate: t0 or h not finite");
  if (!hs::aligned16(c) || !hs::aligned16(ws) || !hs::aligned16(idx_dev) || !hs::aligned16(pot_dev))
    return hs::fail(HS_E_INVALID, "hs_propagate: device pointer not 16-byte aligned");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  for (int64_t n = 0; n < nsteps; ++n) {
    // with t_dev the device clock advances by h per step; without it step n starts at t0 + n h
    const int32_t st = hs::launch_step(idx, idx_dev, pot, pot_dev, dtype, t0 + (double)n * h, t_dev, h, m,
                                       reorth, c, ws, nullptr, s);
    if (st != HS_OK) return st;
  }
  return HS_OK;
}

extern "C" int32_t hs_magnus4_workspace_bytes(hs_index idx, hs_pot pot, int32_t dtype, int32_t m,
                                              int64_t *bytes) {
  if (!idx || !pot || !bytes) return hs::fail(HS_E_INVALID, "hs_magnus4_workspace_bytes: NULL argument");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_magnus4_workspace_bytes: bad dtype");
  if (m < 0 || m > 32) return hs::fail(HS_E_INVALID, "hs_magnus4_workspace_bytes: m out of range 0..32");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_magnus4_workspace_bytes: potential and index differ in N");
  *bytes = m == 0 ? hs::m4_apply_workspace_bytes(idx, pot, dtype) : hs::step4_workspace_bytes(idx, pot, dtype, m);
  return HS_OK;
}

extern "C" int32_t hs_apply_magnus4(hs_index idx, const void *idx_dev, hs_pot pot, const void *pot_dev1,
                                    const void *pot_dev2, int32_t dtype, double h, const void *c, void *y,
                                    void *ws, void *stream) {
  if (!idx || !pot || !idx_dev || !pot_dev1 || !pot_dev2 || !c || !y || !ws)
    return hs::fail(HS_E_INVALID, "hs_apply_magnus4: NULL argument");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_apply_magnus4: potential and index differ in N");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_apply_magnus4: bad dtype");
  if (c == y) return hs::fail(HS_E_INVALID, "hs_apply_magnus4: input and output must differ");
  if (pot_dev1 == pot_dev2) return hs::fail(HS_E_INVALID, "hs_apply_magnus4: the two parameter blocks must differ");
  if (!std::isfinite(h)) return hs::fail(HS_E_NONFINITE, "hs_apply_magnus4: h not finite");
  if (!hs::aligned16(c) || !hs::aligned16(y) || !hs::aligned16(ws) || !hs::aligned16(idx_dev) ||
      !hs::aligned16(pot_dev1) || !hs::aligned16(pot_dev2))
    return hs::fail(HS_E_INVALID, "hs_apply_magnus4: device pointer not 16-byte aligned");
  return hs::launch_apply_m4(idx, idx_dev, pot, pot_dev1, pot_dev2, dtype, h, c, y, ws,
                             static_cast<hipStream_t>(stream));
}

extern "C" int32_t hs_step_magnus4(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev1,
                                   void *pot_dev2, int32_t dtype, double t, double *t_dev, double h,
                                   int32_t m, int32_t reorth, void *c, void *ws, double *diag_dev,
                                   void *stream) {
  if (!idx || !pot || !idx_dev || !pot_dev1 || !pot_dev2 || !c || !ws)
    return hs::fail(HS_E_INVALID, "hs_step_magnus4: NULL argument");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_step_magnus4: potential and index differ in N");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_step_magnus4: bad dtype");
  if (m < 1 || m > 32) return hs::fail(HS_E_INVALID, "hs_step_magnus4: m out of range 1..32");
  if (pot_dev1 == pot_dev2) return hs::fail(HS_E_INVALID, "hs_step_magnus4: the two parameter blocks must differ");
  if (!std::isfinite(h) || (!t_dev && !std::isfinite(t)))
    return hs::fail(HS_E_NONFINITE, "hs_step_magnus4: t or h not finite");
  if (!hs::aligned16(c) || !hs::aligned16(ws) || !hs::aligned16(idx_dev) || !hs::aligned16(pot_dev1) ||
      !hs::aligned16(pot_dev2))
    return hs::fail(HS_E_INVALID, "hs_step_magnus4: device pointer not 16-byte aligned");
  return hs::launch_step_m4(idx, idx_dev, pot, pot_dev1, pot_dev2, dtype, t, t_dev, h, m, reorth, c, ws,
                            diag_dev, static_cast<hipStream_t>(stream));
}
