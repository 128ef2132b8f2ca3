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
#include "matvec_multi.h"

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
// vectors unnormalised: y = s_k H x - beta_{k-1} s_{k-1} prev, s_q = 1 / beta_{q-1}, s_0 = 1.
// One kernel per (N, prefix axes) class, so that each class runs at the occupancy its own
// register count allows; the workgroups of queue q (blocks b with b % kQueues == q) take
// `grab` consecutive work items per atomic increment of that queue's counter.
template <typename T, int N, int NP>
__global__ void __launch_bounds__(256)
k_batch_hh(const BatchInst *__restrict__ insts, const int32_t *__restrict__ items,
           const int64_t *__restrict__ qbeg, int32_t *__restrict__ counters, int32_t grab,
           const typename V2<T>::t *__restrict__ x, typename V2<T>::t *__restrict__ y,
           const typename V2<T>::t *__restrict__ prev, const double *__restrict__ scall, int km1) {
  const int q = blockIdx.x % kQueues;
  const int64_t lo = qbeg[q], hi = qbeg[q + 1];
  const int lane = threadIdx.x & 63;
  constexpr int rs = rec_stride(NP);
  while (true) {
    int32_t got = 0;
    if (lane == 0) got = atomicAdd(&counters[q * 16], grab);  // vector atomic from one lane
    got = __shfl(got, 0);
    if (lo + got >= hi) break;
    for (int32_t g = 0; g < grab; ++g) {
      const int64_t it = lo + got + g;
      if (it >= hi) break;
      const int32_t inst = __builtin_amdgcn_readfirstlane(items[2 * it]);
      const int32_t ch = __builtin_amdgcn_readfirstlane(items[2 * it + 1]);
      const BatchInst &B = insts[inst];
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
      batch_row<T, N, NP>(B, x, y, rec, o, prev, oscale, pcoef);
    }
  }
}

// The long tiles of instances whose potential has no x_l^2 or x_l x_{l+1} monomials, by
// the multi-tile work items of each instance's index set (the single-instance kernel's
// row code, so a batched row equals the single-instance row bit for bit).  Queues and
// grabs as in k_batch_hh; an item is (instance, multi-tile item of that instance).
template <typename T, int N, int NP>
__global__ void __launch_bounds__(256)
k_batch_multi(const BatchInst *__restrict__ insts, const int32_t *__restrict__ items,
              const int64_t *__restrict__ qbeg, int32_t *__restrict__ counters, int32_t grab,
              const typename V2<T>::t *__restrict__ x, typename V2<T>::t *__restrict__ y,
              const typename V2<T>::t *__restrict__ prev, const double *__restrict__ scall, int km1) {
  constexpr int IS = 2 + kMultiTiles;
  const int q = blockIdx.x % kQueues;
  const int64_t lo = qbeg[q], hi = qbeg[q + 1];
  const int lane = threadIdx.x & 63;
  while (true) {
    int32_t got = 0;
    if (lane == 0) got = atomicAdd(&counters[q * 16], grab);  // vector atomic from one lane
    got = __shfl(got, 0);
    if (lo + got >= hi) break;
    for (int32_t g = 0; g < grab; ++g) {
      const int64_t it = lo + got + g;
      if (it >= hi) break;
      const int32_t inst = __builtin_amdgcn_readfirstlane(items[2 * it]);
      const int32_t mi = __builtin_amdgcn_readfirstlane(items[2 * it + 1]);
      const BatchInst &B = insts[inst];
      const double *sI = scall ? scall + (int64_t)inst * Scal::size : nullptr;
      const T oscale = (sI && km1 >= 0) ? (T)sI[Scal::inv + km1] : T(1);
      const T pcoef = (prev && sI) ? (T)(sI[Scal::beta + km1] * (km1 >= 1 ? sI[Scal::inv + km1 - 1] : 1.0)) : T(0);
      multi_item<T, N, NP>(B.ix, B.hh, x + B.off, y + B.off, B.ix.mitems + (int64_t)mi * IS, oscale,
                           prev ? prev + B.off : nullptr, pcoef);
    }
  }
}

// the (N, prefix axes) classes the batched kernels serve, in a fixed order
constexpr int kBatchVariants = 7;
__host__ __device__ constexpr int batch_variant_n(int v) { return v + 2; }
__host__ __device__ constexpr int batch_variant_np(int v) { return v == 0 ? 0 : (v == 1 ? 1 : (v <= 3 ? 2 : v - 1)); }
inline int batch_variant_of(int N, int np) {
  for (int v = 0; v < kBatchVariants; ++v)
    if (batch_variant_n(v) == N && batch_variant_np(v) == np) return v;
  return -1;
}

// kind 0: k_batch_hh over row items; kind 1: k_batch_multi over multi-tile items
template <typename T>
void launch_batch_variant(int kind, int v, unsigned grid, unsigned wg, hipStream_t s, const BatchInst *insts,
                          const int32_t *items, const int64_t *qbeg, int32_t *counters, int32_t grab,
                          const void *x, void *y, const void *prev, const double *sc, int km1) {
  using C = typename V2<T>::t;
#define HS_BV(V)                                                                                        \
  case V:                                                                                               \
    if (kind == 0)                                                                                      \
      hipLaunchKernelGGL((k_batch_hh<T, batch_variant_n(V), batch_variant_np(V)>), dim3(grid), dim3(wg), 0, \
                         s, insts, items, qbeg, counters, grab, (const C *)x, (C *)y, (const C *)prev, sc, km1); \
    else                                                                                                \
      hipLaunchKernelGGL((k_batch_multi<T, batch_variant_n(V), batch_variant_np(V)>), dim3(grid), dim3(wg), 0, \
                         s, insts, items, qbeg, counters, grab, (const C *)x, (C *)y, (const C *)prev, sc, km1); \
    break;
  switch (v) {
    HS_BV(0)
    HS_BV(1)
    HS_BV(2)
    HS_BV(3)
    HS_BV(4)
    HS_BV(5)
    HS_BV(6)
    default:
      break;
  }
#undef HS_BV
}

__global__ void k_batch_reset(int32_t *counters, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i * 16] = 0;
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
  // Work items of the two kernel kinds: kind 0 (k_batch_hh) takes (instance, chunk) pairs,
  // chunk < 0 meaning the short-tile block -chunk-1; kind 1 (k_batch_multi) takes
  // (instance, multi-tile item).  Grouped by kernel class: class v owns
  // [vbeg[kind][v], vbeg[kind][v+1]) of items[kind].
  std::vector<int32_t> items[2];
  std::vector<int64_t> vbeg[2];  // kBatchVariants + 1 each
  std::vector<int64_t> qbeg;     // [kind][class][queue + 1]: queue q owns [qbeg[..][q], qbeg[..][q+1])
  int32_t order = 0;             // 0: largest instances first; 1: instances interleaved
  std::vector<int32_t> seg_inst, seg_len;
  std::vector<int64_t> seg_row0, iseg0;
  int64_t nitems[2] = {0, 0}, nseg = 0;
  int64_t off_insts = 0, off_items[2] = {0, 0}, off_qbeg = 0, off_counters = 0, off_seginst = 0,
          off_segrow0 = 0, off_seglen = 0, off_iseg0 = 0, dev_bytes = 0;
  int32_t wg[2][hs::kBatchVariants], per_cu[2][hs::kBatchVariants], grab[2][hs::kBatchVariants];
  int32_t ncu = 256;             // compute units of the device current at creation
  // the class kernels of one application run concurrently: one side stream per
  // (kind, class), forked from and joined back into the caller's stream by events
  // (default priority; graph capture follows the fork and the join)
  hipStream_t side[2 * hs::kBatchVariants] = {};
  hipEvent_t fork = nullptr, join[2 * hs::kBatchVariants] = {};
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

// Work items of every instance, grouped by kernel class.  An instance whose potential
// has no x_l^2 or x_l x_{l+1} monomials takes its long tiles by multi-tile items (kind 1)
// and its short tiles by 64-row blocks (kind 0), as the single-instance path does;
// otherwise both go to kind 0 (64-row chunks of long tiles, then the short blocks).
// order 0: the largest instances first; order 1: the instances of a class interleaved
// item by item (round robin), so that small and large instances share the queues.  Each
// class's items of each kind are split into one contiguous range per XCD, equal counts.
constexpr size_t qidx(int kind, int v, int q) {
  return ((size_t)kind * hs::kBatchVariants + (size_t)v) * (hs::kQueues + 1) + (size_t)q;
}

static void build_items(hs_batch_s *b, int32_t order) {
  const int n = b->n;
  b->qbeg.assign((size_t)2 * hs::kBatchVariants * (hs::kQueues + 1), 0);
  b->order = order;
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return b->idx[a]->size > b->idx[c]->size; });
  // the same choice as the single-instance path (bit-for-bit equal rows)
  auto multi = [&](int i) { return hs::multi_serves<double>(b->insts[i].ix, b->pot[i]->x2); };
  for (int kind = 0; kind < 2; ++kind) {
    std::vector<int32_t> &items = b->items[kind];
    items.clear();
    b->vbeg[kind].assign(hs::kBatchVariants + 1, 0);
    for (int v = 0; v < hs::kBatchVariants; ++v) {
      const int64_t first = (int64_t)items.size() / 2;
      b->vbeg[kind][v] = first;
      std::vector<int> mine;
      for (int i : ord)
        if (hs::batch_variant_of(b->idx[i]->N, b->idx[i]->np) == v) mine.push_back(i);
      // item k of instance i for this kind
      auto count_of = [&](int i) -> int64_t {
        const hs_index_s *ix = b->idx[i];
        const int64_t shorts = (ix->nsmall + 63) / 64;
        if (kind == 1) return multi(i) ? ix->nmitems : 0;
        return (multi(i) ? 0 : ix->nchunks) + shorts;
      };
      auto push = [&](int i, int64_t k) {
        items.push_back(i);
        if (kind == 1) {
          items.push_back((int32_t)k);
        } else {
          const int64_t nc = multi(i) ? 0 : b->idx[i]->nchunks;
          items.push_back(k < nc ? (int32_t)k : (int32_t)(-(k - nc) - 1));
        }
      };
      if (order == 0) {
        for (int i : mine)
          for (int64_t k = 0; k < count_of(i); ++k) push(i, k);
      } else {
        std::vector<int64_t> next(mine.size(), 0);
        bool any = true;
        while (any) {
          any = false;
          for (size_t j = 0; j < mine.size(); ++j)
            if (next[j] < count_of(mine[j])) {
              push(mine[j], next[j]++);
              any = true;
            }
        }
      }
      const int64_t cnt = (int64_t)items.size() / 2 - first;
      for (int q = 0; q <= hs::kQueues; ++q) b->qbeg[qidx(kind, v, q)] = first + cnt * q / hs::kQueues;
    }
    b->vbeg[kind][hs::kBatchVariants] = (int64_t)items.size() / 2;
    b->nitems[kind] = b->vbeg[kind][hs::kBatchVariants];
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
    for (int kind = 0; kind < 2; ++kind)
      for (int v = 0; v < hs::kBatchVariants; ++v) {
        b->wg[kind][v] = 256;
        b->per_cu[kind][v] = 8;
        b->grab[kind][v] = 1;
      }
    build_items(b, 0);
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
    b->off_items[0] = take(b->nitems[0] * 8);
    b->off_items[1] = take(b->nitems[1] * 8);
    b->off_qbeg = take((int64_t)b->qbeg.size() * 8);
    b->off_counters = take((int64_t)2 * hs::kBatchVariants * hs::kQueues * 64);
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
    put(b->off_items[0], b->items[0].data(), b->nitems[0] * 8);
    put(b->off_items[1], b->items[1].data(), b->nitems[1] * 8);
    put(b->off_qbeg, b->qbeg.data(), (int64_t)b->qbeg.size() * 8);
    put(b->off_seginst, b->seg_inst.data(), b->nseg * 4);
    put(b->off_segrow0, b->seg_row0.data(), b->nseg * 8);
    put(b->off_seglen, b->seg_len.data(), b->nseg * 4);
    put(b->off_iseg0, b->iseg0.data(), (n + 1) * 8);
  } catch (const std::bad_alloc &) {
    delete b;
    return hs::fail(HS_E_NOMEM, "hs_batch_create: out of host memory");
  }
  {
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; i < 2 * hs::kBatchVariants && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      hs_batch_destroy(b);
      return hs::hip_fail(e, "hs_batch_create: side streams");
    }
  }
  *out = b;
  return HS_OK;
}

extern "C" int32_t hs_batch_destroy(hs_batch b) {
  if (!b) return HS_OK;
  for (int i = 0; i < 2 * hs::kBatchVariants; ++i) {
    if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
    if (b->join[i]) (void)hipEventDestroy(b->join[i]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
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
                     const double *sc, int km1, hipStream_t s, int only_kind = -1, int only_v = -1) {
  const int ncu = b->ncu;
  int32_t *counters = (int32_t *)(bd + b->off_counters);
  hipLaunchKernelGGL(hs::k_batch_reset, dim3(1), dim3(256), 0, s, counters, 2 * hs::kBatchVariants * hs::kQueues);
  HS_HIP(hipEventRecord(b->fork, s));
  for (int kind = 0; kind < 2; ++kind) {
    if (only_kind >= 0 && kind != only_kind) continue;
    for (int v = 0; v < hs::kBatchVariants; ++v) {
      if (b->vbeg[kind][v + 1] == b->vbeg[kind][v] || (only_v >= 0 && v != only_v)) continue;
      const int si = kind * hs::kBatchVariants + v;
      hipStream_t ss = b->side[si];
      HS_HIP(hipStreamWaitEvent(ss, b->fork, 0));
      const unsigned grid = hs::xcd_grid((int64_t)ncu * b->per_cu[kind][v]);
      hs::launch_batch_variant<double>(kind, v, grid, (unsigned)b->wg[kind][v], ss,
                                       (const BatchInst *)(bd + b->off_insts),
                                       (const int32_t *)(bd + b->off_items[kind]),
                                       (const int64_t *)(bd + b->off_qbeg) + qidx(kind, v, 0),
                                       counters + ((size_t)kind * hs::kBatchVariants + v) * hs::kQueues * 16,
                                       b->grab[kind][v], x, y, prev, sc, km1);
      HS_HIP(hipEventRecord(b->join[si], ss));
      HS_HIP(hipStreamWaitEvent(s, b->join[si], 0));
    }
  }
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
  for (int kind = 0; kind < 2; ++kind)
    for (int v = 0; v < hs::kBatchVariants; ++v) {
      if (wg) b->wg[kind][v] = wg;
      if (per_cu) b->per_cu[kind][v] = per_cu;
    }
  return HS_OK;
}

// the (kind, class) holding the most work items (its launch is the one reported)
static void main_launch(const hs_batch_s *b, int &kind, int &v) {
  kind = 0;
  v = 0;
  int64_t most = -1;
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < hs::kBatchVariants; ++c) {
      const int64_t cnt = b->vbeg[k][c + 1] - b->vbeg[k][c];
      if (cnt > most) {
        most = cnt;
        kind = k;
        v = c;
      }
    }
}

extern "C" int32_t hs_batch_get_launch(hs_batch b, int32_t *wg, int32_t *per_cu) {
  if (!b) return hs::fail(HS_E_INVALID, "hs_batch_get_launch: NULL handle");
  int kind, v;
  main_launch(b, kind, v);
  if (wg) *wg = b->wg[kind][v];
  if (per_cu) *per_cu = b->per_cu[kind][v];
  return HS_OK;
}

extern "C" int32_t hs_batch_tuning(hs_batch b, int32_t *order, int32_t *table) {
  if (!b || !order || !table) return hs::fail(HS_E_INVALID, "hs_batch_tuning: NULL argument");
  *order = b->order;
  for (int v = 0; v < hs::kBatchVariants; ++v) {
    int32_t *t = table + 10 * v;
    t[0] = hs::batch_variant_n(v);
    t[1] = hs::batch_variant_np(v);
    for (int kind = 0; kind < 2; ++kind) {
      t[2 + 4 * kind] = (int32_t)std::min<int64_t>(b->vbeg[kind][v + 1] - b->vbeg[kind][v], INT32_MAX);
      t[3 + 4 * kind] = b->wg[kind][v];
      t[4 + 4 * kind] = b->per_cu[kind][v];
      t[5 + 4 * kind] = b->grab[kind][v];
    }
  }
  return HS_OK;
}

extern "C" int32_t hs_batch_autotune_sync(hs_batch b, const void *batch_dev, const void *c, void *y,
                                          void *ws, void *stream) {
  if (!b || !batch_dev || !c || !y) return hs::fail(HS_E_INVALID, "hs_batch_autotune_sync: NULL argument");
  (void)ws;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint8_t *bd = static_cast<const uint8_t *>(batch_dev);
  uint8_t *bdw = const_cast<uint8_t *>(bd);
  hipEvent_t e0, e1;
  HS_HIP(hipEventCreate(&e0));
  HS_HIP(hipEventCreate(&e1));
  int32_t st = HS_OK;
  // time of `reps` applications of one (kind, class), or of everything (kind < 0)
  auto timed = [&](int kind, int v, int reps, float &ms) -> int32_t {
    int32_t r = batch_matvec(b, bd, c, y, nullptr, nullptr, 0, s, kind, v);  // warm-up
    if (r != HS_OK) return r;
    if (hipEventRecord(e0, s) != hipSuccess) return hs::fail(HS_E_HIP, "hs_batch_autotune_sync: event record");
    for (int k = 0; k < reps && r == HS_OK; ++k) r = batch_matvec(b, bd, c, y, nullptr, nullptr, 0, s, kind, v);
    if (r != HS_OK) return r;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return hs::fail(HS_E_HIP, "hs_batch_autotune_sync: event synchronisation");
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return hs::fail(HS_E_HIP, "hs_batch_autotune_sync: event time");
    return HS_OK;
  };
  // upload the item lists and queue bounds of the current order (device block and the
  // host image that hs_batch_upload copies)
  auto upload_items = [&]() -> int32_t {
    for (int kind = 0; kind < 2; ++kind) {
      HS_HIP(hipMemcpy(bdw + b->off_items[kind], b->items[kind].data(), b->nitems[kind] * 8, hipMemcpyHostToDevice));
      std::memcpy(b->blob.data() + b->off_items[kind], b->items[kind].data(), b->nitems[kind] * 8);
    }
    HS_HIP(hipMemcpy(bdw + b->off_qbeg, b->qbeg.data(), (int64_t)b->qbeg.size() * 8, hipMemcpyHostToDevice));
    std::memcpy(b->blob.data() + b->off_qbeg, b->qbeg.data(), (int64_t)b->qbeg.size() * 8);
    if (b->pinned) std::memcpy(b->pinned, b->blob.data(), b->dev_bytes);
    return HS_OK;
  };
  const int32_t wgs[3] = {64, 128, 256};
  const int32_t pcs[4] = {2, 4, 8, 16};
  const int32_t grabs[3] = {1, 2, 4};
  float best_order_ms = 1e30f;
  int32_t best_order = b->order;
  int32_t bwg[2][hs::kBatchVariants], bpc[2][hs::kBatchVariants], bgr[2][hs::kBatchVariants];
  for (int order = 0; order < 2 && st == HS_OK; ++order) {
    build_items(b, order);
    st = upload_items();
    // each (kind, class) on its own: workgroup size, workgroups per CU, items per grab
    for (int kind = 0; kind < 2 && st == HS_OK; ++kind)
      for (int v = 0; v < hs::kBatchVariants && st == HS_OK; ++v) {
        if (b->vbeg[kind][v + 1] == b->vbeg[kind][v]) continue;
        float best = 1e30f;
        int32_t w0 = b->wg[kind][v], p0 = b->per_cu[kind][v], g0 = b->grab[kind][v];
        for (int32_t wg : wgs)
          for (int32_t pc : pcs)
            for (int32_t gr : grabs) {
              if (st != HS_OK) break;
              b->wg[kind][v] = wg;
              b->per_cu[kind][v] = pc;
              b->grab[kind][v] = gr;
              float ms = 0.f;
              st = timed(kind, v, 2, ms);
              if (st == HS_OK && ms < best) {
                best = ms;
                w0 = wg;
                p0 = pc;
                g0 = gr;
              }
            }
        b->wg[kind][v] = w0;
        b->per_cu[kind][v] = p0;
        b->grab[kind][v] = g0;
      }
    if (st != HS_OK) break;
    float ms = 0.f;
    st = timed(-1, -1, 3, ms);
    if (st == HS_OK && ms < best_order_ms) {
      best_order_ms = ms;
      best_order = order;
      std::memcpy(bwg, b->wg, sizeof(bwg));
      std::memcpy(bpc, b->per_cu, sizeof(bpc));
      std::memcpy(bgr, b->grab, sizeof(bgr));
    }
  }
  if (st == HS_OK && best_order_ms < 1e30f) {
    std::memcpy(b->wg, bwg, sizeof(bwg));
    std::memcpy(b->per_cu, bpc, sizeof(bpc));
    std::memcpy(b->grab, bgr, sizeof(bgr));
    build_items(b, best_order);
    st = upload_items();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}
