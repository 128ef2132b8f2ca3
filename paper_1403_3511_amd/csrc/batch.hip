// Batched form: many (index set, potential) instances of different N and B advanced
// together.  One persistent launch applies H to every instance: its workgroups pull
// 64-row work items (instance, chunk of a long tile or of the short-tile row list) from
// a device queue and run the compile-time (N, prefix-axes) specialisation of the fused
// row kernel for the item's instance.  The Lanczos vector kernels and the small
// exponentials are the segmented ones of the single-instance step, run over the packed
// vectors of all instances with per-instance scalars.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "lanczos.h"
#include "matvec_long.h"

namespace hs {

int32_t launch_set_time(const hs_pot_s *p, void *pot_dev, double t, const double *t_dev,
                        double dt, hipStream_t s);

struct BatchInst {
  IndexDev ix;                 // device view of the instance's index set
  const double *hh;            // fused coefficients
  const double *base, *amp, *freq, *phase, *M;
  double *beta, *hhw;          // written by the coefficient update
  int32_t nterms, nslots, x2, pad;
  int64_t off;                 // first element of the instance in packed vectors
};

constexpr int kQueues = kXcd;  // one work queue per XCD (L2 locality of an instance)

template <typename T, int N, int NP>
__device__ __forceinline__ void batch_row(const BatchInst &B, const typename V2<T>::t *x,
                                          typename V2<T>::t *y, const int32_t *rec, int32_t o,
                                          const typename V2<T>::t *prev, T oscale, T pcoef) {
  if (B.x2)
    hh_row<T, N, NP, true, false>(B.ix, B.hh, x + B.off, y + B.off, rec, o, oscale, prev ? prev + B.off : nullptr, pcoef);
  else
    hh_row<T, N, NP, false, false>(B.ix, B.hh, x + B.off, y + B.off, rec, o, oscale, prev ? prev + B.off : nullptr, pcoef);
}

// y = H x, or inside a Lanczos step (scall != nullptr, km1 = k - 1 >= 0) with the stored
// vectors unnormalised: y = s_k H x - beta_{k-1} s_{k-1} prev, s_q = 1 / beta_{q-1}, s_0 = 1
template <typename T>
__global__ void __launch_bounds__(256)
k_batch_hh(const BatchInst *__restrict__ insts, const int32_t *__restrict__ items,
           const int64_t *__restrict__ qbeg, int32_t *__restrict__ counters,
           const typename V2<T>::t *__restrict__ x, typename V2<T>::t *__restrict__ y,
           const typename V2<T>::t *__restrict__ prev, const double *__restrict__ scall, int km1) {
  const int q = blockIdx.x % kQueues;
  const int64_t lo = qbeg[q], hi = qbeg[q + 1];
  const int lane = threadIdx.x & 63;
  while (true) {
    int32_t got = 0;
    if (lane == 0) got = atomicAdd(&counters[q * 16], 1);  // vector atomic from one lane
    got = __shfl(got, 0);
    const int64_t it = lo + got;
    if (it >= hi) break;
    const int32_t inst = __builtin_amdgcn_readfirstlane(items[2 * it]);
    const int32_t ch = __builtin_amdgcn_readfirstlane(items[2 * it + 1]);
    const BatchInst &B = insts[inst];
    const int rs = rec_stride(B.ix.np);
    const int32_t *rec;
    int32_t o;
    bool act;
    if (ch >= 0) {
      const int32_t ri = B.ix.chunks[2 * (int64_t)ch];
      rec = B.ix.recs + (int64_t)ri * rs;
      o = B.ix.chunks[2 * (int64_t)ch + 1] + lane;
      act = o < rec[1];
    } else {
      const int64_t i = (int64_t)(-ch - 1) * 64 + lane;
      act = i < B.ix.nsmall;
      const int32_t r = act ? B.ix.small_rows[i] : 0;
      rec = B.ix.recs + (int64_t)B.ix.tile_rec[B.ix.rowtile[r]] * rs;
      o = r - rec[0];
    }
    if (!act) continue;
    const double *sI = scall ? scall + (int64_t)inst * Scal::size : nullptr;
    const T oscale = (sI && km1 >= 0) ? (T)sI[Scal::inv + km1] : T(1);
    const T pcoef = (prev && sI) ? (T)(sI[Scal::beta + km1] * (km1 >= 1 ? sI[Scal::inv + km1 - 1] : 1.0)) : T(0);
    switch (B.ix.N * 32 + B.ix.np) {
#define HS_BCASE(NN, PP) \
  case NN * 32 + PP:     \
    batch_row<T, NN, PP>(B, x, y, rec, o, prev, oscale, pcoef); \
    break;
      HS_BCASE(2, 0)
      HS_BCASE(3, 1)
      HS_BCASE(4, 2)
      HS_BCASE(5, 2)
      HS_BCASE(6, 3)
      HS_BCASE(7, 4)
      HS_BCASE(8, 5)
      default:
        break;
#undef HS_BCASE
    }
  }
}

__global__ void k_batch_reset(int32_t *counters) {
  if (threadIdx.x < kQueues) counters[threadIdx.x * 16] = 0;
}

// beta_t = base_t + amp_t sin(freq_t (t + dt) + phase_t); hh = M beta, per instance
__global__ void k_batch_set_time(const BatchInst *__restrict__ insts, double t_host,
                                 const double *__restrict__ t_dev, double dt) {
  __shared__ double sb[kMaxTerms];
  const BatchInst &B = insts[blockIdx.x];
  const double t = (t_dev ? *t_dev : t_host) + dt;
  for (int i = threadIdx.x; i < B.nterms; i += blockDim.x) {
    const double b = B.base[i] + B.amp[i] * sin(B.freq[i] * t + B.phase[i]);
    sb[i] = b;
    B.beta[i] = b;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < B.nslots; s += blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < B.nterms; ++i) acc = fma(B.M[(int64_t)s * B.nterms + i], sb[i], acc);
    B.hhw[s] = acc;
  }
}

}  // namespace hs

using hs::BatchInst;

struct hs_batch_s {
  int32_t n = 0;
  std::vector<hs_index> idx;
  std::vector<const void *> idx_dev;
  std::vector<hs_pot> pot;
  std::vector<void *> pot_dev;
  std::vector<int64_t> offsets;  // n + 1 element offsets of the packed vectors
  std::vector<BatchInst> insts;
  std::vector<int32_t> items;    // (instance, chunk) pairs; chunk < 0: short-tile block -chunk-1
  std::vector<int64_t> qbeg;     // queue q owns items [qbeg[q], qbeg[q+1])
  std::vector<int32_t> seg_inst, seg_len;
  std::vector<int64_t> seg_row0, iseg0;
  int64_t nitems = 0, nseg = 0;
  int64_t off_insts = 0, off_items = 0, off_qbeg = 0, off_counters = 0, off_seginst = 0,
          off_segrow0 = 0, off_seglen = 0, off_iseg0 = 0, dev_bytes = 0;
  int32_t wg = 256, per_cu = 8;
  int32_t ncu = 256;             // compute units of the device current at creation
  std::vector<uint8_t> blob;
  void *pinned = nullptr;
  hs::SegView view(const void *dev) const {
    const uint8_t *b = static_cast<const uint8_t *>(dev);
    hs::SegView v{};
    v.n = n;
    v.nseg = nseg;
    v.inst = reinterpret_cast<const int32_t *>(b + off_seginst);
    v.row0 = reinterpret_cast<const int64_t *>(b + off_segrow0);
    v.len = reinterpret_cast<const int32_t *>(b + off_seglen);
    v.iseg0 = reinterpret_cast<const int64_t *>(b + off_iseg0);
    v.size = offsets[n];
    return v;
  }
};

static bool batch_supported(int N, int np) {
  switch (N * 32 + np) {
    case 2 * 32 + 0: case 3 * 32 + 1: case 4 * 32 + 2: case 5 * 32 + 2:
    case 6 * 32 + 3: case 7 * 32 + 4: case 8 * 32 + 5:
      return true;
    default:
      return false;
  }
}

extern "C" int32_t hs_batch_create(int32_t n, const hs_index *idx, const void *const *idx_dev,
                                   const hs_pot *pot, void *const *pot_dev, hs_batch *out) {
  if (!out) return hs::fail(HS_E_INVALID, "hs_batch_create: out is NULL");
  *out = nullptr;
  if (n < 1 || !idx || !idx_dev || !pot || !pot_dev) return hs::fail(HS_E_INVALID, "hs_batch_create: bad arguments");
  hs_batch_s *b = new (std::nothrow) hs_batch_s();
  if (!b) return hs::fail(HS_E_NOMEM, "hs_batch_create: out of host memory");
  try {
    b->n = n;
    {
      int dev = 0;
      hipDeviceProp_t pr;
      if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&pr, dev) == hipSuccess)
        b->ncu = pr.multiProcessorCount;
    }
    b->offsets.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      if (!idx[i] || !pot[i] || !idx_dev[i] || !pot_dev[i]) {
        delete b;
        return hs::fail(HS_E_INVALID, "hs_batch_create: NULL instance handle or pointer");
      }
      if (idx[i]->N != pot[i]->N) {
        delete b;
        return hs::fail(HS_E_INVALID, "hs_batch_create: instance potential and index differ in N");
      }
      if (idx[i]->kind != HS_SET_HYPERBOLIC) {
        delete b;
        return hs::fail(HS_E_UNSUPPORTED, "hs_batch_create: batches serve hyperbolic sets only");
      }
      if (pot[i]->form != HS_FORM_PAPER) {
        delete b;
        return hs::fail(HS_E_UNSUPPORTED, "hs_batch_create: batches serve the paper's operator form only");
      }
      if (!pot[i]->fused || !idx[i]->recs_all || !batch_supported(idx[i]->N, idx[i]->np)) {
        delete b;
        return hs::fail(HS_E_UNSUPPORTED, "hs_batch_create: instance outside the batched kernel's classes "
                                          "(fused potential, default tile dimension, N in 2..8)");
      }
      b->idx.push_back(idx[i]);
      b->idx_dev.push_back(idx_dev[i]);
      b->pot.push_back(pot[i]);
      b->pot_dev.push_back(pot_dev[i]);
      b->offsets[i + 1] = b->offsets[i] + hs::align_up(idx[i]->size, 64);
    }
    if (b->offsets[n] >= (INT64_C(1) << 31)) {
      delete b;
      return hs::fail(HS_E_OVERFLOW, "hs_batch_create: 2^31 or more rows in the batch");
    }
    // instance descriptors
    b->insts.resize(n);
    for (int i = 0; i < n; ++i) {
      BatchInst &B = b->insts[i];
      std::memset(&B, 0, sizeof(B));
      B.ix = idx[i]->view(idx_dev[i]);
      const uint8_t *pb = static_cast<const uint8_t *>(pot_dev[i]);
      const hs_pot_s *p = pot[i];
      B.hh = (const double *)(pb + p->off_hh);
      B.base = (const double *)(pb + p->off_base);
      B.amp = (const double *)(pb + p->off_amp);
      B.freq = (const double *)(pb + p->off_freq);
      B.phase = (const double *)(pb + p->off_phase);
      B.M = (const double *)(pb + p->off_M);
      B.beta = (double *)(pb + p->off_beta);
      B.hhw = (double *)(pb + p->off_hh);
      B.nterms = p->nterms;
      B.nslots = p->nslots;
      B.x2 = p->x2 ? 1 : 0;
      B.off = b->offsets[i];
    }
    // work items, largest instances first, split into one queue per XCD with equal counts
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return idx[a]->size > idx[c]->size; });
    for (int i : order) {
      for (int64_t ch = 0; ch < idx[i]->nchunks; ++ch) {
        b->items.push_back(i);
        b->items.push_back((int32_t)ch);
      }
      for (int64_t k = 0; k * 64 < idx[i]->nsmall; ++k) {
        b->items.push_back(i);
        b->items.push_back((int32_t)(-k - 1));
      }
    }
    b->nitems = (int64_t)b->items.size() / 2;
    b->qbeg.resize(hs::kQueues + 1);
    for (int q = 0; q <= hs::kQueues; ++q) b->qbeg[q] = b->nitems * q / hs::kQueues;
    // segments
    b->iseg0.push_back(0);
    for (int i = 0; i < n; ++i) {
      for (int64_t r = 0; r < idx[i]->size; r += hs::kSeg) {
        b->seg_inst.push_back(i);
        b->seg_row0.push_back(b->offsets[i] + r);
        b->seg_len.push_back((int32_t)std::min<int64_t>(hs::kSeg, idx[i]->size - r));
      }
      b->iseg0.push_back((int64_t)b->seg_inst.size());
    }
    b->nseg = (int64_t)b->seg_inst.size();
    // device image
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
      int64_t o = off;
      off = hs::align_up(off + std::max<int64_t>(bytes, 1), 256);
      return o;
    };
    b->off_insts = take((int64_t)sizeof(BatchInst) * n);
    b->off_items = take(b->nitems * 8);
    b->off_qbeg = take((hs::kQueues + 1) * 8);
    b->off_counters = take(hs::kQueues * 64);
    b->off_seginst = take(b->nseg * 4);
    b->off_segrow0 = take(b->nseg * 8);
    b->off_seglen = take(b->nseg * 4);
    b->off_iseg0 = take((n + 1) * 8);
    b->dev_bytes = off;
    b->blob.assign(off, 0);
    auto put = [&](int64_t o, const void *src, int64_t bytes) {
      if (bytes > 0) std::memcpy(b->blob.data() + o, src, bytes);
    };
    put(b->off_insts, b->insts.data(), (int64_t)sizeof(BatchInst) * n);
    put(b->off_items, b->items.data(), b->nitems * 8);
    put(b->off_qbeg, b->qbeg.data(), (hs::kQueues + 1) * 8);
    put(b->off_seginst, b->seg_inst.data(), b->nseg * 4);
    put(b->off_segrow0, b->seg_row0.data(), b->nseg * 8);
    put(b->off_seglen, b->seg_len.data(), b->nseg * 4);
    put(b->off_iseg0, b->iseg0.data(), (n + 1) * 8);
  } catch (const std::bad_alloc &) {
    delete b;
    return hs::fail(HS_E_NOMEM, "hs_batch_create: out of host memory");
  }
  *out = b;
  return HS_OK;
}

extern "C" int32_t hs_batch_destroy(hs_batch b) {
  if (!b) return HS_OK;
  if (b->pinned) (void)hipHostFree(b->pinned);
  delete b;
  return HS_OK;
}

extern "C" int32_t hs_batch_offsets(hs_batch b, int64_t *host_out) {
  if (!b || !host_out) return hs::fail(HS_E_INVALID, "hs_batch_offsets: NULL argument");
  std::memcpy(host_out, b->offsets.data(), (b->n + 1) * sizeof(int64_t));
  return HS_OK;
}

extern "C" int32_t hs_batch_device_bytes(hs_batch b, int64_t *bytes) {
  if (!b || !bytes) return hs::fail(HS_E_INVALID, "hs_batch_device_bytes: NULL argument");
  *bytes = b->dev_bytes;
  return HS_OK;
}

extern "C" int32_t hs_batch_upload(hs_batch b, void *dev, int64_t bytes, void *stream) {
  if (!b || !dev) return hs::fail(HS_E_INVALID, "hs_batch_upload: NULL argument");
  if (bytes < b->dev_bytes) return hs::fail(HS_E_WORKSPACE, "hs_batch_upload: device buffer too small");
  if (reinterpret_cast<uintptr_t>(dev) % 16) return hs::fail(HS_E_INVALID, "hs_batch_upload: device pointer not 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!b->pinned) {
    HS_HIP(hipHostMalloc(&b->pinned, b->dev_bytes, hipHostMallocDefault));
    std::memcpy(b->pinned, b->blob.data(), b->dev_bytes);
  }
  HS_HIP(hipMemcpyAsync(dev, b->pinned, b->dev_bytes, hipMemcpyHostToDevice, s));
  return HS_OK;
}

extern "C" int32_t hs_batch_workspace_bytes(hs_batch b, int32_t m, int64_t *bytes) {
  if (!b || !bytes) return hs::fail(HS_E_INVALID, "hs_batch_workspace_bytes: NULL argument");
  if (m < 0 || m > hs::kMaxM) return hs::fail(HS_E_INVALID, "hs_batch_workspace_bytes: m out of range 0..32");
  *bytes = m == 0 ? 0 : hs::step_layout(b->offsets[b->n], b->nseg, b->n, 16, m, 0).total;
  return HS_OK;
}

namespace {

int32_t batch_matvec(hs_batch_s *b, const uint8_t *bd, const void *x, void *y, const void *prev,
                     const double *sc, int km1, hipStream_t s) {
  const int ncu = b->ncu;
  int32_t *counters = (int32_t *)(bd + b->off_counters);
  hipLaunchKernelGGL(hs::k_batch_reset, dim3(1), dim3(64), 0, s, counters);
  const unsigned grid = hs::xcd_grid((int64_t)ncu * b->per_cu);
  hipLaunchKernelGGL(hs::k_batch_hh<double>, dim3(grid), dim3(b->wg), 0, s,
                     (const BatchInst *)(bd + b->off_insts), (const int32_t *)(bd + b->off_items),
                     (const int64_t *)(bd + b->off_qbeg), counters, (const double2 *)x, (double2 *)y,
                     (const double2 *)prev, sc, km1);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

// the batched kernel evaluates the paper's operator form; a form set on an instance's
// potential after the batch was created is refused here rather than ignored
int32_t check_forms(const hs_batch_s *b, const char *who) {
  for (const hs_pot_s *p : b->pot)
    if (p->form != HS_FORM_PAPER)
      return hs::fail(HS_E_UNSUPPORTED, std::string(who) + ": an instance's potential is not in the paper's form");
  return HS_OK;
}

}  // namespace

extern "C" int32_t hs_batch_apply_h(hs_batch b, const void *batch_dev, const void *c, void *y,
                                    void *ws, void *stream) {
  (void)ws;
  if (!b || !batch_dev || !c || !y) return hs::fail(HS_E_INVALID, "hs_batch_apply_h: NULL argument");
  if (c == y) return hs::fail(HS_E_INVALID, "hs_batch_apply_h: input and output must differ");
  if (int32_t st = check_forms(b, "hs_batch_apply_h")) return st;
  return batch_matvec(b, static_cast<const uint8_t *>(batch_dev), c, y, nullptr, nullptr, 0,
                      static_cast<hipStream_t>(stream));
}

extern "C" int32_t hs_batch_step(hs_batch b, void *batch_dev, double t, double *t_dev, double h,
                                 int32_t m, int32_t reorth, void *c, void *ws, void *stream) {
  if (!b || !batch_dev || !c || !ws) return hs::fail(HS_E_INVALID, "hs_batch_step: NULL argument");
  if (m < 1 || m > hs::kMaxM) return hs::fail(HS_E_INVALID, "hs_batch_step: m out of range 1..32");
  if (!std::isfinite(h) || (!t_dev && !std::isfinite(t))) return hs::fail(HS_E_NONFINITE, "hs_batch_step: t or h not finite");
  if (int32_t st = check_forms(b, "hs_batch_step")) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint8_t *bd = static_cast<const uint8_t *>(batch_dev);
  hs::StepJob J;
  J.rows = b->offsets[b->n];
  J.sv = b->view(batch_dev);
  J.apply_ws = 0;
  J.set_time = [&](hipStream_t st) {
    hipLaunchKernelGGL(hs::k_batch_set_time, dim3(b->n), dim3(256), 0, st,
                       (const BatchInst *)(bd + b->off_insts), t, (const double *)t_dev, 0.5 * h);
    HS_HIP(hipGetLastError());
    return (int32_t)HS_OK;
  };
  J.matvec = [&](const void *vk, void *w, const void *vprev, int k, double *sc, void *, hipStream_t st) {
    return batch_matvec(b, bd, vk, w, vprev, sc, k - 1, st);
  };
  return hs::run_step<double>(J, m, reorth, h, c, ws, t_dev, t_dev, nullptr, s);
}

extern "C" int32_t hs_batch_set_launch(hs_batch b, int32_t wg, int32_t per_cu) {
  if (!b) return hs::fail(HS_E_INVALID, "hs_batch_set_launch: NULL handle");
  if (wg != 0 && wg != 64 && wg != 128 && wg != 256) return hs::fail(HS_E_INVALID, "hs_batch_set_launch: wg must be 64, 128 or 256");
  if (per_cu < 0 || per_cu > 64) return hs::fail(HS_E_INVALID, "hs_batch_set_launch: per_cu out of range 0..64");
  if (wg) b->wg = wg;
  if (per_cu) b->per_cu = per_cu;
  return HS_OK;
}

extern "C" int32_t hs_batch_get_launch(hs_batch b, int32_t *wg, int32_t *per_cu) {
  if (!b) return hs::fail(HS_E_INVALID, "hs_batch_get_launch: NULL handle");
  if (wg) *wg = b->wg;
  if (per_cu) *per_cu = b->per_cu;
  return HS_OK;
}

extern "C" int32_t hs_batch_autotune_sync(hs_batch b, const void *batch_dev, const void *c, void *y,
                                          void *ws, void *stream) {
  if (!b || !batch_dev || !c || !y) return hs::fail(HS_E_INVALID, "hs_batch_autotune_sync: NULL argument");
  (void)ws;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HS_HIP(hipEventCreate(&e0));
  HS_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int32_t bwg = b->wg, bpc = b->per_cu;
  const int32_t wgs[3] = {64, 128, 256};
  const int32_t pcs[4] = {2, 4, 8, 16};
  int32_t st = HS_OK;
  for (int32_t wg : wgs)
    for (int32_t pc : pcs) {
      b->wg = wg;
      b->per_cu = pc;
      st = batch_matvec(b, static_cast<const uint8_t *>(batch_dev), c, y, nullptr, nullptr, 0, s);
      if (st != HS_OK) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 3 && st == HS_OK; ++r)
        st = batch_matvec(b, static_cast<const uint8_t *>(batch_dev), c, y, nullptr, nullptr, 0, s);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) st = HS_E_HIP;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (st == HS_OK && ms < best) {
        best = ms;
        bwg = wg;
        bpc = pc;
      }
      if (st != HS_OK) break;
    }
  b->wg = bwg;
  b->per_cu = bpc;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}
