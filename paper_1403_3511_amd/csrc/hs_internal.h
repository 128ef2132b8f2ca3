// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hs.h"

namespace hs {

// ---- error reporting ----------------------------------------------------------------
void set_error(const std::string &msg);
int32_t fail(int32_t code, const std::string &msg);
int32_t hip_fail(hipError_t e, const char *what);
#define HS_HIP(call)                                             \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return ::hs::hip_fail(e_, #call);      \
  } while (0)

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// ---- index set ------------------------------------------------------------------------
// Device view of the tiled index layout.  All arrays live in one caller buffer.
struct IndexDev {
  int32_t N, d, np;          // dimension, suffix axes per tile, prefix axes (N - d)
  int32_t B;                 // product bound
  int64_t size;              // |K|
  int64_t ntiles, ng;        // tiles, entries of the global suffix list
  const int64_t *tstart;     // [ntiles + 1] first row of each tile
  const int32_t *tlen;       // [ntiles]
  const int32_t *tnbr;       // [ntiles][2 np]: 2l -> prefix - e_l, 2l+1 -> prefix + e_l (-1: none)
  const uint16_t *tpfx;      // [ntiles][np] prefix multi-index
  const int32_t *tpsum;      // [ntiles] sum of prefix coordinates
  const uint16_t *gsidx;     // [ng][d] suffix multi-index (graded order)
  const int32_t *gnbr;       // [ng][2d]: 2a -> s - e_a, 2a+1 -> s + e_a (-1: not in K_d(B))
  const int32_t *gssum;      // [ng] sum of suffix coordinates
  const int32_t *rowtile;    // [size] tile of each row
  const double *wtab;        // [B + 8] sqrt(k / 2)
  const float *wtabf;        // [B + 8] sqrt(k / 2) in float32
  const double *wtp;         // [B + 10] sqrt((k - 2) / 2) for k >= 2, 0 below (window loads)
  const float *wtpf;         // the same in float32
  const uint64_t *gsp;       // [ng] suffix multi-index packed 16 bits per axis (d <= 4), else NULL
  // suffix stencil (graded offset of s(o) + displacement, or -1), stored in pairs that the
  // fused kernel reads together: gst[2 (p ng + o) + side], see gst_axis_at / gst_cross_at
  int32_t ns;                // number of entries per suffix = 6 d + 8 (d - 1)
  const int32_t *gst;
  // work lists of the fused kernel
  int64_t nchunks;           // 64-row chunks of the long tiles: (record, first offset)
  const int32_t *chunks;     // [nchunks][2]
  int32_t rstride;           // int32 per long-tile record
  const int32_t *recs;       // long-tile records (layout: see rec_* below)
  const int32_t *tile_rec;   // [ntiles] record of every tile, or NULL (long tiles only)
  int64_t nsmall;            // rows of the short tiles
  const int32_t *small_rows; // [nsmall]
  // work items of the multi-tile kernel: (first offset, tile count, kMultiTiles records)
  int64_t nmitems;
  const int32_t *mitems;     // [nmitems][2 + kMultiTiles]
  uint32_t *dbg;             // [2] failed neighbour-index checks of the debug build, first code
};

// Suffix stencil pairs.  Axis pairs p = 3 a + (|s| - 1) hold the displacements -|s|
// (side 0) and +|s| (side 1) along suffix axis a, |s| = 1..3.  Cross pairs
// p = 3 d + 4 a + i(s) hold s along a and r = -1 (side 0) / +1 (side 1) along a + 1, for
// s in {-2, -1, 1, 2}.
__host__ __device__ inline int gst_axis_pair(int a, int sabs) { return 3 * a + sabs - 1; }
__host__ __device__ inline int gst_cross_pair(int d, int a, int s) {
  return 3 * d + 4 * a + (s < 0 ? s + 2 : s + 1);
}
__host__ __device__ inline int64_t gst_elem(int pair, int side, int64_t o, int64_t ng) {
  return 2 * ((int64_t)pair * ng + o) + side;
}
__host__ __device__ inline int64_t gst_axis_at(int a, int s, int64_t o, int64_t ng) {
  return gst_elem(gst_axis_pair(a, s < 0 ? -s : s), s > 0 ? 1 : 0, o, ng);
}
__host__ __device__ inline int64_t gst_cross_at(int d, int a, int s, int r, int64_t o, int64_t ng) {
  return gst_elem(gst_cross_pair(d, a, s), r > 0 ? 1 : 0, o, ng);
}
// Long-tile record (int32): [0] first row, [1] length, [2] sum of prefix coordinates,
// [3] tile id, [4 .. 4+np) prefix coordinates, then (first row, length) pairs of the
// neighbour tiles the two-axis stencil reaches: for each prefix axis l the tiles
// p + s e_l, s in {-3,-2,-1,1,2,3}; for each prefix pair (l, l+1) the tiles
// p + s e_l + r e_{l+1}, s in {-2..2}, r in {-1,1}.  Absent tiles have length 0.
__host__ __device__ constexpr int rec_stride(int np) { return 4 + np + 2 * (6 * np + 10 * (np > 1 ? np - 1 : 0)); }
__host__ __device__ constexpr int rec_axis(int np, int l, int s) {
  return 4 + np + 2 * (l * 6 + (s < 0 ? s + 3 : s + 2));
}
__host__ __device__ constexpr int rec_pair(int np, int l, int s, int r) {
  return 4 + np + 2 * (6 * np + l * 10 + (s + 2) * 2 + (r > 0 ? 1 : 0));
}
constexpr int kChunk = 64;       // rows per wave in the long-tile kernel
constexpr int kMultiTiles = 4;   // tiles per work item of the multi-tile kernel
constexpr int kLongTile = 32;    // tiles at least this long go to the long-tile kernel
// Fibres for chained recurrence passes (hs_index_build_fibres): positions per batch (one
// workgroup of kFibBatch threads, one position each), and the longest chain, which is
// also the halo kept on each side of a fibre segment.
constexpr int kFibBatch = 256;
constexpr int kChainMax = 8;
constexpr int kFibCore = kFibBatch - 2 * kChainMax;  // most core positions of one segment
constexpr int kCombChains = 8;  // most chains fused with a combination

}  // namespace hs

struct hs_index_s {
  int32_t N = 0, d = 0, np = 0;
  int64_t B = 0, size = 0, ntiles = 0, ng = 0;
  int32_t kind = HS_SET_HYPERBOLIC;   // HS_SET_BOX: {0..kmax}^N; HS_SET_TOTAL_DEGREE: |k|_1 <= deg;
                                      // HS_SET_LIST: an explicit downward-closed set;
                                      // HS_SET_PADDED: prod(1 + max(k - deg, 0)) <= B - deg
  int64_t kmax = 0, deg = 0;
  std::shared_ptr<struct ListSet> list;  // HS_SET_LIST rows (index.cpp)
  std::vector<uint16_t> tpfx;
  std::vector<int64_t> tstart;
  std::vector<int32_t> tlen, tnbr, tpsum;
  std::vector<uint16_t> gsidx;
  std::vector<int32_t> gnbr, gssum;
  std::vector<int32_t> rowtile;
  std::vector<int32_t> gst, chunks, small_rows, recs, tile_rec, mitems;
  int32_t ns = 0, rstride = 0;
  bool recs_all = false;
  int64_t nchunks = 0, nsmall = 0, nmitems = 0;
  // device blob layout (byte offsets)
  int64_t off_tstart = 0, off_tlen = 0, off_tnbr = 0, off_tpfx = 0, off_tpsum = 0,
          off_gsidx = 0, off_gnbr = 0, off_gssum = 0, off_rowtile = 0, off_wtab = 0,
          off_wtabf = 0, off_wtp = 0, off_wtpf = 0, off_gsp = 0, off_gst = 0, off_chunks = 0, off_small = 0, off_recs = 0, off_tile_rec = 0, off_mitems = 0, off_dbg = 0,
          dev_bytes = 0;
  std::vector<uint8_t> blob;   // host image of the device block
  void *pinned = nullptr;      // pinned staging for the upload
  // fibres along every axis (hs_index_build_fibres), appended to the device block:
  // positions row | fibre coordinate << 32 | flags << 48, the distances of each position to
  // its k - 1 and k + 1 positions (16 bits each), and batch starts (nb + 1 per axis)
  bool fibres = false;
  bool fibres_uploaded = false;             // the last upload carried them (kernels use them then)
  int64_t off_fpos = 0, off_fdel = 0, off_fbat = 0;
  std::vector<int64_t> fpos0, fbat0, fnb;   // per axis: first position, first batch entry, batches
  hs::IndexDev view(const void *dev) const;
};

namespace hs {

// ---- potential ----------------------------------------------------------------------
constexpr int kMaxTerms = 512;

// Fused class-HH kernel parameters: per outer axis l
//   t_l = X_l ( X_l ( X_l (a3 c) + g2 X_{l+1} c + a2 c ) + g1 X_{l+1} c + a1 c ) + g0' ...
// stored as coefficients of the monomials x_l^a (a = 1..3) and x_l^a x_{l+1} (a = 0..2).
struct HHCoef {
  double a[HS_NMAX][4];   // a[l][p]: coefficient of x_l^p (p = 1..3)
  double g[HS_NMAX][3];   // g[l][p]: coefficient of x_l^p x_{l+1} (p = 0..2)
  double c0;              // constant
};

// Generic program of recurrence passes over whole vectors.
// Program step over whole vectors (slot 0: input, slot 1: output y, others workspace).
//  kind 0: dst = A X_axis(src) + Bc src - C prev + plus   (prev, plus optional)
//  kind 1: y += coef * src
//  kind 2: the combination W_o = sum_e beta[term_e] V_{in_e} (tables in the potential)
// For kinds 0 and 1, term >= 0 accumulates beta[term] * (result) into y; term == -2
// accumulates it with coefficient 1; term == -1 does not accumulate.
constexpr int kTermOne = -2;
struct PassOp {
  int32_t kind;
  int32_t axis;      // axis for kind 0
  int32_t src, prev, dst;  // vector slots (-1 none)
  double A, Bc, C;   // recurrence coefficients
  int32_t term;
  int32_t plus;      // kind 0: slot added to the result (-1 none)
};
constexpr int kMaxComb = 64;  // inputs / outputs of the combination step
constexpr int kCombRegs = 32; // most inputs of the combination held in registers per row

}  // namespace hs

struct hs_pot_s {
  int32_t N = 0, basis = 0, nterms = 0;
  double scale = 1.0;
  std::vector<uint16_t> deg;          // nterms x N
  std::vector<double> base, amp, freq, phase;
  bool fused = false;
  bool x2 = false;                    // fused form uses x_l^2 or x_l x_{l+1} monomials
  bool x2_struct = false;             // ... for some choice of the coefficients
  bool dyn_linear = false;            // time-dependent terms reach only x_l^1 and constant slots
  int32_t form = HS_FORM_PAPER;       // operator form (hs_pot_set_form)
  // fused: compiled monomial coefficient of each HH slot = sum_t M[slot][t] beta_t
  int32_t nslots = 0;
  std::vector<double> M;              // nslots x nterms
  // generic program
  std::vector<hs::PassOp> prog;
  // chains of recurrence passes along one axis (op i + 1 continues op i's recurrence):
  // chain[i] = steps of the chain that starts at op i (1: a pass of its own, 0: inside a
  // chain); keep[i] = whether op i's output is read after its chain
  std::vector<int32_t> chain;
  std::vector<uint8_t> keep;
  // the split program's combination fused with the chains that follow it along one axis
  // (ops [cg_op, cg_end), on sets with fibres): combination outputs whose value is read
  // after those chains are written through (cg_wt, combination output indices)
  int32_t cg_op = -1, cg_end = -1;
  std::vector<int32_t> cg_wt;
  // consecutive independent chains along one axis run as one launch: mc_end[i] = the end
  // of the group that starts at op i (0: none)
  std::vector<int32_t> mc_end;
  int32_t nslots_vec = 0;             // vector slots used by the program
  int32_t split = 0;                  // outer axes evaluated by Clenshaw sums (0: trie only)
  // combination step (split > 0): output o = sum over entries e in [cptr[o], cptr[o+1])
  // of beta[cterm[e]] * slot cin_slot[cidx[e]]
  std::vector<int32_t> cin_slot, cout_slot, cptr, cidx, cterm;
  // device block: beta[kMaxTerms] | base | amp | freq | phase | M | hh coefficients
  int64_t dev_bytes = 0;
  int64_t off_beta = 0, off_base = 0, off_amp = 0, off_freq = 0, off_phase = 0, off_M = 0,
          off_hh = 0, off_comb = 0;
};

namespace hs {
int32_t compile_potential(hs_pot_s *p);
// kernels (implemented in the .hip translation units)
int32_t launch_set_time(const hs_pot_s *p, void *pot_dev, double t, const double *t_dev,
                        double dt_offset, hipStream_t s);
// y = out_scale * H x - prev_coef * prev_scale * prev (the optional terms when non-NULL)
int32_t launch_apply(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p,
                     const void *pot_dev, int32_t dtype, const void *x, void *y, void *ws,
                     hipStream_t s, const double *out_scale, const void *prev,
                     const double *prev_coef, const double *prev_scale);
int32_t launch_apply_x(const hs_index_s *idx, const void *idx_dev, int32_t axis, int32_t dtype,
                       const void *x, void *y, hipStream_t s);
int64_t apply_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype);
// The exact Galerkin operator D + W_{K,pol} on the rows of sub, as the fast algorithm on a
// padded set pad restricted to sub (complex128; map = hs_index_embed(sub, pad) on the device):
// y = out_scale * Omega(F_pad Omega_+(x)) - prev_coef * prev_scale * prev (diag.hip)
int64_t exact_apply_workspace_bytes(const hs_index_s *pad, const hs_pot_s *p);
int32_t launch_exact_apply(const hs_index_s *sub, const hs_index_s *pad, const void *pad_dev, const int32_t *map,
                           const hs_pot_s *p, const void *pot_dev, const void *x, void *y, void *ws, hipStream_t s,
                           const double *out_scale, const void *prev, const double *prev_coef,
                           const double *prev_scale);
// one exponential-midpoint step with that operator (lanczos.hip)
int32_t launch_step_exact(const hs_index_s *sub, const hs_index_s *pad, const void *pad_dev, const int32_t *map,
                          const hs_pot_s *p, void *pot_dev, double t, double *t_dev, double h, int m, int reorth,
                          void *c, void *ws, double *diag, hipStream_t s);
int64_t step_exact_workspace_bytes(const hs_index_s *sub, const hs_index_s *pad, const hs_pot_s *p, int m);
// row limit of the one-workgroup step (0: never)
void set_small_step_rows(int64_t rows);
int64_t small_step_rows();
}  // namespace hs
