// Host-side construction of the tiled index layout of K_N(B) = {k : prod(1 + k_l) <= B}
// (paper Sec. 1.2) with the neighbour maps k +- e_l needed by the direct operation with
// the coordinate matrices (Sec. 3.1).
//
// Layout.  Rows are grouped into tiles sharing the prefix p = (k_1..k_{N-d}).  The tile
// of p has remaining bound b_p = floor(B / prod(1 + p_i)); its rows are the suffixes
// s in K_d(b_p).  All suffix lists are initial segments of ONE global list G = K_d(B)
// sorted by (prod(1 + s), lex s), so the row (p, s) sits at tstart[p] + pos_G(s) and a
// move along a prefix axis keeps the offset inside the tile.
#include <algorithm>
#include <memory>
#include <string>
#include <unordered_map>
#include <cstring>
#include <new>

#include "hs_internal.h"

// An explicit downward-closed set (HS_SET_LIST).  For N >= 3 (and N = 1) its tiles are the
// distinct prefixes (first N - 1 coordinates) and the suffix is the last coordinate: by
// downward closure every fibre is {0..L-1}, an initial segment of the one suffix list
// {0..maxlen-1}, so the tiled layout and its fused kernels apply.  For N = 2 every axis
// is a prefix axis: one row per tile, the empty suffix.
struct ListSet {
  int N = 0;
  int d = 0;                                       // tile dimension: 0 (one row per tile) or 1
  std::vector<uint16_t> k;                         // rows, lexicographic
  std::unordered_map<std::string, int64_t> pos;    // key -> row
  // d = 1: the distinct prefixes (first N - 1 coordinates, lexicographic), the length of
  // each one's fibre along the last axis (downward closure makes it {0..L-1}), and the
  // longest fibre
  std::vector<uint16_t> pfx;
  std::vector<int32_t> flen;
  std::unordered_map<std::string, int64_t> ppos;   // prefix key -> prefix index
  int32_t maxlen = 0;
  static std::string key(const int32_t *m, int n) {
    std::string s((size_t)n * 2, '\0');
    for (int i = 0; i < n; ++i) {
      s[2 * i] = (char)(m[i] & 0xFF);
      s[2 * i + 1] = (char)((m[i] >> 8) & 0xFF);
    }
    return s;
  }
};

namespace {

constexpr int64_t kSat = INT64_C(1) << 62;

// a + f * c for non-negative terms, saturating at kSat (counts of large padded crosses
// exceed 64 bits: 17^16 rows at N = 16, w = 16)
inline int64_t sat_fma(int64_t a, int64_t f, int64_t c) {
  if (f != 0 && c > (kSat - a) / f) return kSat;
  return a + f * c;
}

// Coordinate cost of the product-bound sets: 1 + k on the hyperbolic cross, and on the
// padded cross 1 + max(k - w, 0), so that the values 0..w all cost 1.
inline int64_t pcost(int64_t k, int64_t w) { return 1 + (k > w ? k - w : 0); }

// |K_n(b)| for every b in the set {floor(B / q)} that division keeps reaching (with pad
// width w: the padded cross prod(1 + max(k_l - w, 0)) <= b).
struct Counter {
  int64_t B = 0, w = 0;
  int nmax = 0;
  std::vector<int32_t> slot;                 // b -> position in vals (-1: unreachable)
  std::vector<int64_t> vals;                 // reachable bounds, ascending
  std::vector<std::vector<int64_t>> cnt;     // cnt[n][slot]
  Counter(int64_t B_, int nmax_, int64_t w_ = 0) : B(B_), w(w_), nmax(nmax_), slot(B_ + 1, -1) {
    for (int64_t q = 1; q <= B; ++q) {
      int64_t b = B / q;
      if (slot[b] < 0) slot[b] = 0;
      if (b * b < B && q * q >= B) {  // remaining values are exactly 1..b
        for (int64_t x = 1; x <= b; ++x) slot[x] = 0;
        break;
      }
    }
    for (int64_t b = 1; b <= B; ++b)
      if (slot[b] >= 0) {
        slot[b] = (int32_t)vals.size();
        vals.push_back(b);
      }
    cnt.assign(nmax + 1, std::vector<int64_t>(vals.size(), 0));
    for (size_t i = 0; i < vals.size(); ++i) cnt[0][i] = 1;
    for (int n = 1; n <= nmax; ++n)
      for (size_t i = 0; i < vals.size(); ++i) {
        int64_t b = vals[i], s = 0;
        // group the terms a with equal floor(b / a)
        for (int64_t a = 1; a <= b;) {
          int64_t v = b / a, a2 = b / v;
          s = sat_fma(s, a2 - a + 1, cnt[n - 1][slot[v]]);
          a = a2 + 1;
        }
        // the w further values of cost 1 on the padded cross
        s = sat_fma(s, w, cnt[n - 1][slot[b]]);
        cnt[n][i] = s;
      }
  }
  int64_t count(int n, int64_t b) const { return b < 1 ? 0 : cnt[n][slot[b]]; }
};

// Lexicographic rank inside K_n(B) for multi-indices of length n.
struct LexRank {
  const Counter *C;
  int n;
  int64_t B;
  // cum[i][slot(b)][a] = sum_{a' < a} |K_{n-1-i}(floor(b / cost(a')))|
  std::vector<std::vector<std::vector<int64_t>>> cum;
  LexRank(const Counter *C_, int n_, int64_t B_) : C(C_), n(n_), B(B_) {
    cum.resize(n);
    for (int i = 0; i < n; ++i) {
      cum[i].resize(C->vals.size());
      for (size_t si = 0; si < C->vals.size(); ++si) {
        int64_t b = C->vals[si];
        auto &v = cum[i][si];
        v.resize(b + C->w + 1);  // values 0 .. b - 1 + w have cost <= b
        v[0] = 0;
        for (int64_t a = 0; a < b + C->w; ++a) v[a + 1] = v[a] + C->count(n - 1 - i, b / pcost(a, C->w));
      }
    }
  }
  // k must be a member
  int64_t rank(const int32_t *k) const {
    int64_t r = 0, b = B;
    for (int i = 0; i < n; ++i) {
      r += cum[i][C->slot[b]][k[i]];
      b /= pcost(k[i], C->w);
    }
    return r;
  }
};

bool member(const int32_t *k, int n, int64_t B, int64_t w = 0) {
  int64_t p = 1;
  for (int i = 0; i < n; ++i) {
    if (k[i] < 0) return false;
    p *= pcost(k[i], w);
    if (p > B) return false;
  }
  return true;
}

// Lexicographic enumeration of K_n(B) (with pad width w: of the padded cross): calls f(k)
// for each member.
template <class F>
void enumerate(int n, int64_t B, F &&f, int64_t w = 0) {
  std::vector<int32_t> k(n, 0);
  if (n == 0) {
    f(k.data());
    return;
  }
  std::vector<int64_t> bound(n + 1);
  bound[0] = B;
  int lvl = 0;
  k[0] = 0;
  while (true) {
    // descend with zeros
    for (; lvl < n - 1; ++lvl) {
      bound[lvl + 1] = bound[lvl] / pcost(k[lvl], w);
      k[lvl + 1] = 0;
    }
    // at the last level run over all admissible values
    int64_t b = bound[n - 1];
    for (int32_t a = 0; a < b + w; ++a) {
      k[n - 1] = a;
      f(k.data());
    }
    // advance the deepest level that can still grow
    int up = n - 2;
    while (up >= 0) {
      k[up] += 1;
      if (pcost(k[up], w) <= bound[up]) break;
      --up;
    }
    if (up < 0) return;
    lvl = up;
  }
}

// Lexicographic enumeration of the box {0..K}^n.
template <class F>
void enumerate_box(int n, int64_t K, F &&f) {
  std::vector<int32_t> k(n, 0);
  while (true) {
    f(k.data());
    int i = n - 1;
    while (i >= 0 && k[i] == K) k[i--] = 0;
    if (i < 0) return;
    ++k[i];
  }
}

// Lexicographic enumeration of the simplex {k : |k|_1 <= D}.
template <class F>
void enumerate_simplex(int n, int64_t D, F &&f) {
  std::vector<int32_t> k(n, 0);
  int64_t sum = 0;
  while (true) {
    f(k.data());
    int i = n - 1;
    // raise the deepest coordinate that still fits, clearing the ones after it
    while (i >= 0 && sum >= D) {
      sum -= k[i];
      k[i] = 0;
      --i;
    }
    if (i < 0) return;
    ++k[i];
    ++sum;
  }
}

// |{k in N_0^n : |k|_1 <= b}| = C(n + b, n), saturated
int64_t simplex_count(int n, int64_t b) {
  if (b < 0) return 0;
  double c = 1.0;
  for (int i = 1; i <= n; ++i) c = c * (double)(b + i) / i;
  return c > (double)kSat ? kSat : (int64_t)(c + 0.5);
}

// The set the layout is built for, as a budget that the coordinates spend:
//   hyperbolic cross prod(1 + k_l) <= B  (grade of a suffix: prod(1 + s_a));
//   box {0..K}^n                          (one grade);
//   total degree |k|_1 <= D               (grade: |s|_1).
// A tile with prefix p keeps the suffixes whose grade fits the budget p leaves, and
// these are an initial segment of the suffix list sorted by (grade, lex): that is what
// lets a move along a prefix axis keep the row's offset inside the tile.
struct SetOps {
  int kind = HS_SET_HYPERBOLIC;
  int64_t B = 0, K = 0, D = 0;
  std::unique_ptr<Counter> C;
  const ListSet *L = nullptr;
  // B: product bound (hyperbolic and padded); K: box edge; D: total degree, or the pad
  // width w of the padded cross
  SetOps(int kind_, int64_t B_, int64_t K_, int64_t D_, int N, const ListSet *L_ = nullptr)
      : kind(kind_), B(B_), K(K_), D(D_), L(L_) {
    if (product()) C.reset(new Counter(B, N, pad()));
  }
  bool product() const { return kind == HS_SET_HYPERBOLIC || kind == HS_SET_PADDED; }
  int64_t pad() const { return kind == HS_SET_PADDED ? D : 0; }
  // Lists with tile dimension 1 answer prefix queries (n = N - 1) from the fibres and
  // suffix queries (n = 1) with {0..maxlen-1}; N >= 3 there, so the two never coincide.
  int64_t count(int n) const {
    if (kind == HS_SET_LIST) {
      if (n == 0) return 1;
      if (n == L->N) return (int64_t)L->pos.size();
      return n == 1 ? L->maxlen : (int64_t)L->flen.size();
    }
    if (product()) return C->count(n, B);
    if (kind == HS_SET_TOTAL_DEGREE) return simplex_count(n, D);
    int64_t r = 1;
    for (int i = 0; i < n; ++i) r = sat_fma(0, r, K + 1);
    return r;
  }
  bool member(const int32_t *k, int n) const {
    if (kind == HS_SET_LIST) {
      if (n == 0) return true;
      for (int i = 0; i < n; ++i)
        if (k[i] < 0 || k[i] > 65535) return false;
      if (n == L->N) return L->pos.count(ListSet::key(k, n)) > 0;
      if (n == 1) return k[0] < L->maxlen;
      return L->ppos.count(ListSet::key(k, n)) > 0;
    }
    if (product()) return ::member(k, n, B, pad());
    int64_t sum = 0;
    for (int i = 0; i < n; ++i) {
      if (k[i] < 0 || (kind == HS_SET_BOX && k[i] > K)) return false;
      sum += k[i];
    }
    return kind == HS_SET_BOX || sum <= D;
  }
  template <class F> void each(int n, F &&f) const {
    if (kind == HS_SET_LIST) {
      std::vector<int32_t> m(n);
      if (n == 0) {
        f(m.data());
        return;
      }
      if (n == L->N) {
        const int64_t rows = (int64_t)L->pos.size();
        for (int64_t r = 0; r < rows; ++r) {
          for (int i = 0; i < n; ++i) m[i] = L->k[(size_t)r * n + i];
          f(m.data());
        }
      } else if (n == 1) {
        for (int32_t a = 0; a < L->maxlen; ++a) {
          m[0] = a;
          f(m.data());
        }
      } else {
        const int64_t np = (int64_t)L->flen.size();
        for (int64_t t = 0; t < np; ++t) {
          for (int i = 0; i < n; ++i) m[i] = L->pfx[(size_t)t * n + i];
          f(m.data());
        }
      }
      return;
    }
    if (kind == HS_SET_BOX) enumerate_box(n, K, f);
    else if (kind == HS_SET_TOTAL_DEGREE) enumerate_simplex(n, D, f);
    else enumerate(n, B, f, pad());
  }
  int64_t grade(const int32_t *s, int d) const {
    if (kind == HS_SET_LIST) return d == 1 ? s[0] : 0;  // a fibre is {0..L-1}
    if (kind == HS_SET_BOX) return 0;
    int64_t g = product() ? 1 : 0;
    for (int a = 0; a < d; ++a) g = product() ? g * pcost(s[a], pad()) : g + s[a];
    return g;
  }
  int64_t max_grade() const {
    if (kind == HS_SET_LIST) return L->d == 1 ? L->maxlen - 1 : 0;
    return product() ? B : (kind == HS_SET_TOTAL_DEGREE ? D : 0);
  }
  // largest suffix grade that fits after prefix p
  int64_t budget(const int32_t *p, int np) const {
    if (kind == HS_SET_LIST) return L->d == 1 ? L->flen[L->ppos.at(ListSet::key(p, np))] - 1 : 0;
    if (kind == HS_SET_BOX) return 0;
    if (kind == HS_SET_TOTAL_DEGREE) {
      int64_t sum = 0;
      for (int i = 0; i < np; ++i) sum += p[i];
      return D - sum;
    }
    int64_t prod = 1;
    for (int i = 0; i < np; ++i) prod *= pcost(p[i], pad());
    return B / prod;
  }
};

// Lexicographic rank among the members of dimension n.
struct Ranker {
  const SetOps *S;
  int n;
  std::unique_ptr<LexRank> R;
  Ranker(const SetOps *S_, int n_) : S(S_), n(n_) {
    if (S->product()) R.reset(new LexRank(S->C.get(), n, S->B));
  }
  int64_t rank(const int32_t *k) const {
    if (S->kind == HS_SET_LIST) {
      if (n == 0) return 0;
      if (n == S->L->N) return S->L->pos.at(ListSet::key(k, n));
      return n == 1 ? k[0] : S->L->ppos.at(ListSet::key(k, n));
    }
    if (S->product()) return R->rank(k);
    int64_t r = 0;
    if (S->kind == HS_SET_BOX) {
      for (int i = 0; i < n; ++i) r = r * (S->K + 1) + k[i];
      return r;
    }
    int64_t left = S->D;  // members before k: those that differ first at position i below k_i
    for (int i = 0; i < n; ++i) {
      for (int32_t a = 0; a < k[i]; ++a) r += simplex_count(n - 1 - i, left - a);
      left -= k[i];
    }
    return r;
  }
};

}  // namespace

hs::IndexDev hs_index_s::view(const void *dev) const {
  const uint8_t *b = static_cast<const uint8_t *>(dev);
  hs::IndexDev v;
  v.N = N;
  v.d = d;
  v.np = np;
  v.B = (int32_t)B;
  v.size = size;
  v.ntiles = ntiles;
  v.ng = ng;
  v.tstart = reinterpret_cast<const int64_t *>(b + off_tstart);
  v.tlen = reinterpret_cast<const int32_t *>(b + off_tlen);
  v.tnbr = reinterpret_cast<const int32_t *>(b + off_tnbr);
  v.tpfx = reinterpret_cast<const uint16_t *>(b + off_tpfx);
  v.tpsum = reinterpret_cast<const int32_t *>(b + off_tpsum);
  v.gsidx = reinterpret_cast<const uint16_t *>(b + off_gsidx);
  v.gnbr = reinterpret_cast<const int32_t *>(b + off_gnbr);
  v.gssum = reinterpret_cast<const int32_t *>(b + off_gssum);
  v.rowtile = reinterpret_cast<const int32_t *>(b + off_rowtile);
  v.wtab = reinterpret_cast<const double *>(b + off_wtab);
  v.wtabf = reinterpret_cast<const float *>(b + off_wtabf);
  v.wtp = reinterpret_cast<const double *>(b + off_wtp);
  v.wtpf = reinterpret_cast<const float *>(b + off_wtpf);
  v.gsp = d <= 4 ? reinterpret_cast<const uint64_t *>(b + off_gsp) : nullptr;
  v.ns = ns;
  v.gst = reinterpret_cast<const int32_t *>(b + off_gst);
  v.nchunks = nchunks;
  v.chunks = reinterpret_cast<const int32_t *>(b + off_chunks);
  v.nsmall = nsmall;
  v.small_rows = reinterpret_cast<const int32_t *>(b + off_small);
  v.rstride = rstride;
  v.recs = reinterpret_cast<const int32_t *>(b + off_recs);
  v.tile_rec = recs_all ? reinterpret_cast<const int32_t *>(b + off_tile_rec) : nullptr;
  v.nmitems = nmitems;
  v.mitems = reinterpret_cast<const int32_t *>(b + off_mitems);
  v.dbg = const_cast<uint32_t *>(reinterpret_cast<const uint32_t *>(b + off_dbg));
  return v;
}

// The set operations of an index handle (padded crosses keep B = product bound + w as
// their coordinate bound, and w in deg).
static SetOps set_ops(const hs_index_s *ix) {
  const int64_t pb = ix->kind == HS_SET_PADDED ? ix->B - ix->deg : ix->B;
  return SetOps(ix->kind, pb, ix->kmax, ix->deg, ix->N, ix->list.get());
}

static int32_t default_tile_dim(int32_t N) { return N <= 2 ? N : (N <= 4 ? 2 : (N <= 8 ? 3 : 4)); }

static int32_t build_index(hs_index_s *ix) {
  const int N = ix->N, d = ix->d, np = ix->np;
  const int64_t B = ix->B;  // coordinates stay below B (weight tables)
  const SetOps S = set_ops(ix);
  const int64_t total = S.count(N);
  if (total >= (INT64_C(1) << 31) - 1) return hs::fail(HS_E_OVERFLOW, "index set has 2^31 or more rows");
  const int64_t ntiles = S.count(np);
  const int64_t ng = S.count(d);
  ix->size = total;
  ix->ntiles = ntiles;
  ix->ng = ng;

  // ---- global suffix list G = K_d(B), graded by (prod, lex) ----
  std::vector<int32_t> glex((size_t)ng * d);
  std::vector<int64_t> gprod(ng);
  {
    int64_t i = 0;
    S.each(d, [&](const int32_t *k) {
      for (int a = 0; a < d; ++a) glex[i * d + a] = k[a];
      gprod[i] = S.grade(k, d);
      ++i;
    });
  }
  std::vector<int64_t> order(ng);
  for (int64_t i = 0; i < ng; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return gprod[a] < gprod[b]; });
  std::vector<int64_t> gpos_of_lex(ng);
  for (int64_t g = 0; g < ng; ++g) gpos_of_lex[order[g]] = g;
  ix->gsidx.resize((size_t)ng * d);
  ix->gssum.resize(ng);
  for (int64_t g = 0; g < ng; ++g) {
    int32_t s = 0;
    for (int a = 0; a < d; ++a) {
      ix->gsidx[g * d + a] = (uint16_t)glex[order[g] * d + a];
      s += glex[order[g] * d + a];
    }
    ix->gssum[g] = s;
  }
  // length of the initial segment with grade <= b
  std::vector<int32_t> seglen(S.max_grade() + 1, 0);
  for (int64_t g = 0; g < ng; ++g) seglen[gprod[order[g]]]++;
  for (int64_t b = 1; b <= S.max_grade(); ++b) seglen[b] += seglen[b - 1];
  // suffix neighbours
  ix->gnbr.assign((size_t)ng * 2 * d, -1);
  if (d > 0) {
    Ranker R(&S, d);
    std::vector<int32_t> k(d);
    for (int64_t g = 0; g < ng; ++g) {
      for (int a = 0; a < d; ++a) k[a] = ix->gsidx[g * d + a];
      for (int a = 0; a < d; ++a)
        for (int dir = 0; dir < 2; ++dir) {
          k[a] += dir ? 1 : -1;
          if (S.member(k.data(), d)) ix->gnbr[g * 2 * d + 2 * a + dir] = (int32_t)gpos_of_lex[R.rank(k.data())];
          k[a] -= dir ? 1 : -1;
        }
    }
  }

  // ---- tiles: prefixes K_np(B) in lex order ----
  ix->tpfx.resize((size_t)ntiles * np);
  ix->tlen.resize(ntiles);
  ix->tpsum.resize(ntiles);
  ix->tstart.resize(ntiles + 1);
  {
    int64_t t = 0, start = 0;
    S.each(np, [&](const int32_t *p) {
      int64_t prod = 1;
      int32_t s = 0;
      for (int i = 0; i < np; ++i) {
        ix->tpfx[t * np + i] = (uint16_t)p[i];
        prod *= 1 + p[i];
        s += p[i];
      }
      ix->tlen[t] = seglen[S.budget(p, np)];
      ix->tpsum[t] = s;
      ix->tstart[t] = start;
      start += ix->tlen[t];
      ++t;
    });
    ix->tstart[ntiles] = start;
    if (start != total) return hs::fail(HS_E_INVALID, "internal: tile lengths do not add up to |K|");
  }
  ix->tnbr.assign((size_t)ntiles * 2 * np, -1);
  if (np > 0) {
    Ranker R(&S, np);
    std::vector<int32_t> p(np);
    for (int64_t t = 0; t < ntiles; ++t) {
      for (int i = 0; i < np; ++i) p[i] = ix->tpfx[t * np + i];
      for (int i = 0; i < np; ++i)
        for (int dir = 0; dir < 2; ++dir) {
          p[i] += dir ? 1 : -1;
          if (S.member(p.data(), np)) ix->tnbr[t * 2 * np + 2 * i + dir] = (int32_t)R.rank(p.data());
          p[i] -= dir ? 1 : -1;
        }
    }
  }
  ix->rowtile.resize(total);
  for (int64_t t = 0; t < ntiles; ++t)
    for (int64_t r = ix->tstart[t]; r < ix->tstart[t + 1]; ++r) ix->rowtile[r] = (int32_t)t;

  // ---- suffix stencil (displacements used by the fused two-axis kernel) ----
  ix->ns = d > 0 ? 6 * d + 8 * (d - 1) : 0;
  ix->gst.assign((size_t)ix->ns * ng, -1);
  if (d > 0) {
    Ranker R(&S, d);
    std::vector<int32_t> k(d);
    auto lookup = [&](int64_t g, int a, int s, int b, int r) -> int32_t {
      for (int i = 0; i < d; ++i) k[i] = ix->gsidx[g * d + i];
      k[a] += s;
      if (b >= 0) k[b] += r;
      if (!S.member(k.data(), d)) return -1;
      return (int32_t)gpos_of_lex[R.rank(k.data())];
    };
    for (int64_t g = 0; g < ng; ++g) {
      for (int a = 0; a < d; ++a)
        for (int s = -3; s <= 3; ++s)
          if (s != 0) ix->gst[hs::gst_axis_at(a, s, g, ng)] = lookup(g, a, s, -1, 0);
      for (int a = 0; a + 1 < d; ++a)
        for (int s : {-2, -1, 1, 2})
          for (int r : {-1, 1}) ix->gst[hs::gst_cross_at(d, a, s, r, g, ng)] = lookup(g, a, s, a + 1, r);
    }
  }
  // ---- work lists: 64-row chunks of long tiles, rows of short tiles ----
  ix->chunks.clear();
  ix->small_rows.clear();
  ix->recs.clear();
  ix->rstride = hs::rec_stride(np);
  auto walk = [&](int64_t t, int l, int s) -> int64_t {  // tile p + s e_l or -1
    for (int k = 0; k < (s < 0 ? -s : s) && t >= 0; ++k) t = ix->tnbr[t * 2 * np + 2 * l + (s > 0)];
    return t;
  };
  // records for every tile when they cost at most 96 bytes per row (then the short
  // tiles use them too), else for the long tiles only
  const int64_t nlong = std::count_if(ix->tlen.begin(), ix->tlen.end(), [](int32_t l) { return l >= hs::kLongTile; });
  // (at most 8 GB in any case: beyond that the short tiles take the row kernel)
  ix->recs_all = (int64_t)ix->rstride * 4 * ntiles <= std::min<int64_t>(
                     std::max<int64_t>(total * 96, INT64_C(64) << 20), INT64_C(8) << 30);
  ix->recs.reserve((size_t)ix->rstride * (ix->recs_all ? ntiles : nlong));
  ix->tile_rec.assign(ix->recs_all ? ntiles : 0, -1);
  for (int64_t t = 0; t < ntiles; ++t) {
    const int32_t len = ix->tlen[t];
    if (len >= hs::kLongTile || ix->recs_all) {
      const int32_t ri = (int32_t)(ix->recs.size() / ix->rstride);
      if (ix->recs_all) ix->tile_rec[t] = ri;
      ix->recs.resize(ix->recs.size() + ix->rstride, 0);
      int32_t *rec = ix->recs.data() + (size_t)ri * ix->rstride;
      rec[0] = (int32_t)ix->tstart[t];
      rec[1] = len;
      rec[2] = ix->tpsum[t];
      rec[3] = (int32_t)t;
      for (int i = 0; i < np; ++i) rec[4 + i] = ix->tpfx[t * np + i];
      auto put = [&](int pos, int64_t tt) {
        rec[pos] = tt >= 0 ? (int32_t)ix->tstart[tt] : 0;
        rec[pos + 1] = tt >= 0 ? ix->tlen[tt] : 0;
      };
      for (int l = 0; l < np; ++l)
        for (int s : {-3, -2, -1, 1, 2, 3}) put(hs::rec_axis(np, l, s), walk(t, l, s));
      for (int l = 0; l + 1 < np; ++l)
        for (int s = -2; s <= 2; ++s)
          for (int r : {-1, 1}) {
            // p + s e_l + r e_{l+1} may exist when p + s e_l does not (r = -1): then walk
            // along l + 1 first (the symmetrised operator reads such tiles)
            int64_t tt = walk(t, l, s);
            int64_t u = tt >= 0 ? walk(tt, l + 1, r) : -1;
            if (u < 0) {
              const int64_t t2 = walk(t, l + 1, r);
              u = t2 >= 0 ? walk(t2, l, s) : -1;
            }
            put(hs::rec_pair(np, l, s, r), u);
          }
      if (len >= hs::kLongTile)
        for (int32_t o = 0; o < len; o += hs::kChunk) {
          ix->chunks.push_back(ri);
          ix->chunks.push_back(o);
        }
    }
    if (len < hs::kLongTile) {
      for (int32_t o = 0; o < len; ++o) ix->small_rows.push_back((int32_t)(ix->tstart[t] + o));
    }
  }
  ix->nchunks = (int64_t)ix->chunks.size() / 2;
  ix->nsmall = (int64_t)ix->small_rows.size();

  // ---- work items of the multi-tile kernel: for each 64-offset range, the long tiles
  // reaching into it, in tile order, kMultiTilesHost at a time (longest first inside an
  // item); items ordered by their first tile, so that each XCD's contiguous share of
  // items covers a contiguous range of tiles ----
  ix->mitems.clear();
  {
    constexpr int R = hs::kMultiTiles, IS = 2 + R;
    std::vector<std::pair<int64_t, int32_t>> longt;  // (tile, record) of the long tiles
    {
      int32_t ri = 0;
      for (int64_t t = 0; t < ntiles; ++t) {
        const int32_t len = ix->tlen[t];
        if (ix->recs_all) {
          if (len >= hs::kLongTile) longt.emplace_back(t, ix->tile_rec[t]);
        } else if (len >= hs::kLongTile) {
          longt.emplace_back(t, ri++);
        }
      }
    }
    int32_t maxlen = 0;
    for (auto &pr : longt) maxlen = std::max(maxlen, ix->tlen[pr.first]);
    const int64_t nblk = maxlen / hs::kChunk + 1;
    // reach[b]: the long tiles (indices into longt, in tile order) longer than b * kChunk
    std::vector<std::vector<int32_t>> reach((size_t)nblk);
    for (size_t i = 0; i < longt.size(); ++i)
      for (int32_t o0 = 0; o0 < ix->tlen[longt[i].first]; o0 += hs::kChunk)
        reach[o0 / hs::kChunk].push_back((int32_t)i);
    std::vector<std::pair<int64_t, std::vector<int32_t>>> items;  // (sort key, item words)
    for (int64_t b = 0; b < nblk; ++b) {
      const std::vector<int32_t> &rb = reach[(size_t)b];
      for (size_t a = 0; a < rb.size(); a += R) {
        const size_t nr = std::min<size_t>(R, rb.size() - a);
        std::vector<int32_t> grp(rb.begin() + a, rb.begin() + a + nr);
        std::stable_sort(grp.begin(), grp.end(), [&](int32_t u, int32_t v) {
          return ix->tlen[longt[u].first] > ix->tlen[longt[v].first];
        });
        std::vector<int32_t> w(IS, 0);
        w[0] = (int32_t)(b * hs::kChunk);
        w[1] = (int32_t)nr;
        for (size_t q = 0; q < nr; ++q) w[2 + q] = longt[grp[q]].second;
        for (size_t q = nr; q < (size_t)R; ++q) w[2 + q] = w[2];
        items.emplace_back(longt[rb[a]].first * nblk + b, std::move(w));
      }
      std::vector<int32_t>().swap(reach[(size_t)b]);
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const auto &u, const auto &v) { return u.first < v.first; });
    ix->mitems.reserve(items.size() * IS);
    for (auto &it : items) ix->mitems.insert(ix->mitems.end(), it.second.begin(), it.second.end());
    ix->nmitems = (int64_t)items.size();
  }

  // ---- device image ----
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off = hs::align_up(off + std::max<int64_t>(bytes, 1), 256);
    return o;
  };
  ix->off_tstart = take((ntiles + 1) * 8);
  ix->off_tlen = take(ntiles * 4);
  ix->off_tnbr = take(ntiles * 2 * np * 4);
  ix->off_tpfx = take(ntiles * np * 2);
  ix->off_tpsum = take(ntiles * 4);
  ix->off_gsidx = take(ng * d * 2);
  ix->off_gnbr = take(ng * 2 * d * 4);
  ix->off_gssum = take(ng * 4);
  ix->off_rowtile = take(total * 4);
  ix->off_wtab = take((B + 8) * 8);
  ix->off_wtabf = take((B + 8) * 4);
  ix->off_wtp = take((B + 10) * 8);
  ix->off_wtpf = take((B + 10) * 4);
  ix->off_gsp = take(d <= 4 ? ng * 8 : 0);
  ix->off_gst = take((int64_t)ix->ns * ng * 4);
  ix->off_chunks = take(ix->nchunks * 8);
  ix->off_small = take(ix->nsmall * 4);
  ix->off_recs = take((int64_t)ix->recs.size() * 4);
  ix->off_tile_rec = take((int64_t)ix->tile_rec.size() * 4);
  ix->off_mitems = take((int64_t)ix->mitems.size() * 4);
  ix->off_dbg = take(8);  // the debug build's check counters, zero on upload
  ix->dev_bytes = off;
  ix->blob.assign(off, 0);
  auto put = [&](int64_t o, const void *src, int64_t bytes) {
    if (bytes > 0) std::memcpy(ix->blob.data() + o, src, bytes);
  };
  put(ix->off_tstart, ix->tstart.data(), (ntiles + 1) * 8);
  put(ix->off_tlen, ix->tlen.data(), ntiles * 4);
  put(ix->off_tnbr, ix->tnbr.data(), ntiles * 2 * np * 4);
  put(ix->off_tpfx, ix->tpfx.data(), ntiles * np * 2);
  put(ix->off_tpsum, ix->tpsum.data(), ntiles * 4);
  put(ix->off_gsidx, ix->gsidx.data(), ng * d * 2);
  put(ix->off_gnbr, ix->gnbr.data(), ng * 2 * d * 4);
  put(ix->off_gssum, ix->gssum.data(), ng * 4);
  put(ix->off_rowtile, ix->rowtile.data(), total * 4);
  std::vector<double> w(B + 8);
  std::vector<float> wf(B + 8);
  for (int64_t k = 0; k < B + 8; ++k) {
    w[k] = std::sqrt(0.5 * (double)k);
    wf[k] = (float)w[k];
  }
  put(ix->off_wtab, w.data(), (B + 8) * 8);
  put(ix->off_wtabf, wf.data(), (B + 8) * 4);
  std::vector<double> wp(B + 10, 0.0);
  std::vector<float> wpf(B + 10, 0.0f);
  for (int64_t k = 2; k < B + 10; ++k) {
    wp[k] = std::sqrt(0.5 * (double)(k - 2));
    wpf[k] = (float)wp[k];
  }
  put(ix->off_wtp, wp.data(), (B + 10) * 8);
  put(ix->off_wtpf, wpf.data(), (B + 10) * 4);
  if (d <= 4) {
    std::vector<uint64_t> pk(ng, 0);
    for (int64_t g = 0; g < ng; ++g)
      for (int a = 0; a < d; ++a) pk[g] |= (uint64_t)ix->gsidx[g * d + a] << (16 * a);
    put(ix->off_gsp, pk.data(), ng * 8);
  }
  put(ix->off_gst, ix->gst.data(), (int64_t)ix->ns * ng * 4);
  put(ix->off_chunks, ix->chunks.data(), ix->nchunks * 8);
  put(ix->off_small, ix->small_rows.data(), ix->nsmall * 4);
  put(ix->off_recs, ix->recs.data(), (int64_t)ix->recs.size() * 4);
  put(ix->off_tile_rec, ix->tile_rec.data(), (int64_t)ix->tile_rec.size() * 4);
  put(ix->off_mitems, ix->mitems.data(), (int64_t)ix->mitems.size() * 4);
  return HS_OK;
}

extern "C" int32_t hs_index_create(int32_t N, int64_t B, int32_t tile_dim, hs_index *out) {
  if (!out) return hs::fail(HS_E_INVALID, "hs_index_create: out is NULL");
  *out = nullptr;
  if (N < 1 || N > HS_NMAX) return hs::fail(HS_E_INVALID, "hs_index_create: N out of range 1..16");
  if (B < 1 || B > 65536) return hs::fail(HS_E_INVALID, "hs_index_create: B out of range 1..65536");
  if (tile_dim < 0 || tile_dim > N) return hs::fail(HS_E_INVALID, "hs_index_create: tile_dim out of range 0..N");
  hs_index_s *ix = new (std::nothrow) hs_index_s();
  if (!ix) return hs::fail(HS_E_NOMEM, "hs_index_create: out of host memory");
  ix->N = N;
  ix->B = B;
  ix->d = tile_dim ? tile_dim : default_tile_dim(N);
  ix->np = N - ix->d;
  int32_t st;
  try {
    st = build_index(ix);
  } catch (const std::bad_alloc &) {
    st = hs::fail(HS_E_NOMEM, "hs_index_create: out of host memory");
  }
  if (st != HS_OK) {
    delete ix;
    return st;
  }
  *out = ix;
  return HS_OK;
}

extern "C" int32_t hs_index_count(int32_t N, int64_t B, int64_t *n) {
  if (!n) return hs::fail(HS_E_INVALID, "hs_index_count: n is NULL");
  *n = 0;
  if (N < 1 || N > HS_NMAX) return hs::fail(HS_E_INVALID, "hs_index_count: N out of range 1..16");
  if (B < 1 || B > 65536) return hs::fail(HS_E_INVALID, "hs_index_count: B out of range 1..65536");
  try {
    Counter C(B, N);
    *n = C.count(N, B);
  } catch (const std::bad_alloc &) {
    return hs::fail(HS_E_NOMEM, "hs_index_count: out of host memory");
  }
  return HS_OK;
}

extern "C" int32_t hs_index_create_box(int32_t N, int64_t Kmax, int32_t tile_dim, hs_index *out) {
  if (!out) return hs::fail(HS_E_INVALID, "hs_index_create_box: out is NULL");
  *out = nullptr;
  if (N < 1 || N > HS_NMAX) return hs::fail(HS_E_INVALID, "hs_index_create_box: N out of range 1..16");
  if (Kmax < 0 || Kmax > 65535) return hs::fail(HS_E_INVALID, "hs_index_create_box: Kmax out of range 0..65535");
  if (tile_dim < 0 || tile_dim > N) return hs::fail(HS_E_INVALID, "hs_index_create_box: tile_dim out of range 0..N");
  int64_t total = 1;
  for (int i = 0; i < N; ++i) {
    total *= Kmax + 1;
    if (total >= (INT64_C(1) << 31) - 1) return hs::fail(HS_E_OVERFLOW, "hs_index_create_box: 2^31 or more rows");
  }
  hs_index_s *ix = new (std::nothrow) hs_index_s();
  if (!ix) return hs::fail(HS_E_NOMEM, "hs_index_create_box: out of host memory");
  ix->N = N;
  ix->kind = HS_SET_BOX;
  ix->kmax = Kmax;
  ix->B = Kmax + 1;  // coordinates stay below B, as on a hyperbolic set with bound B
  ix->d = tile_dim ? tile_dim : default_tile_dim(N);
  ix->np = N - ix->d;
  int32_t st;
  try {
    st = build_index(ix);
  } catch (const std::bad_alloc &) {
    st = hs::fail(HS_E_NOMEM, "hs_index_create_box: out of host memory");
  }
  if (st != HS_OK) {
    delete ix;
    return st;
  }
  *out = ix;
  return HS_OK;
}

extern "C" int32_t hs_index_create_padded(int32_t N, int64_t B, int64_t w, int32_t tile_dim, hs_index *out) {
  if (!out) return hs::fail(HS_E_INVALID, "hs_index_create_padded: out is NULL");
  *out = nullptr;
  if (N < 1 || N > HS_NMAX) return hs::fail(HS_E_INVALID, "hs_index_create_padded: N out of range 1..16");
  if (w < 0 || w > 16) return hs::fail(HS_E_INVALID, "hs_index_create_padded: w out of range 0..16");
  if (B < 1 || B + w > 65536) return hs::fail(HS_E_INVALID, "hs_index_create_padded: need 1 <= B and B + w <= 65536");
  if (tile_dim < 0 || tile_dim > N) return hs::fail(HS_E_INVALID, "hs_index_create_padded: tile_dim out of range 0..N");
  {
    Counter C(B, N, w);
    if (C.count(N, B) >= (INT64_C(1) << 31) - 1) return hs::fail(HS_E_OVERFLOW, "hs_index_create_padded: 2^31 or more rows");
  }
  hs_index_s *ix = new (std::nothrow) hs_index_s();
  if (!ix) return hs::fail(HS_E_NOMEM, "hs_index_create_padded: out of host memory");
  ix->N = N;
  ix->kind = HS_SET_PADDED;
  ix->deg = w;
  ix->B = B + w;  // coordinates stay below B + w
  ix->d = tile_dim ? tile_dim : default_tile_dim(N);
  ix->np = N - ix->d;
  int32_t st;
  try {
    st = build_index(ix);
  } catch (const std::bad_alloc &) {
    st = hs::fail(HS_E_NOMEM, "hs_index_create_padded: out of host memory");
  }
  if (st != HS_OK) {
    delete ix;
    return st;
  }
  *out = ix;
  return HS_OK;
}

extern "C" int32_t hs_index_create_total_degree(int32_t N, int64_t D, int32_t tile_dim, hs_index *out) {
  if (!out) return hs::fail(HS_E_INVALID, "hs_index_create_total_degree: out is NULL");
  *out = nullptr;
  if (N < 1 || N > HS_NMAX) return hs::fail(HS_E_INVALID, "hs_index_create_total_degree: N out of range 1..16");
  if (D < 0 || D > 65535) return hs::fail(HS_E_INVALID, "hs_index_create_total_degree: D out of range 0..65535");
  if (tile_dim < 0 || tile_dim > N) return hs::fail(HS_E_INVALID, "hs_index_create_total_degree: tile_dim out of range 0..N");
  if (simplex_count(N, D) >= (INT64_C(1) << 31) - 1)
    return hs::fail(HS_E_OVERFLOW, "hs_index_create_total_degree: 2^31 or more rows");
  hs_index_s *ix = new (std::nothrow) hs_index_s();
  if (!ix) return hs::fail(HS_E_NOMEM, "hs_index_create_total_degree: out of host memory");
  ix->N = N;
  ix->kind = HS_SET_TOTAL_DEGREE;
  ix->deg = D;
  ix->B = D + 1;  // coordinates stay below B, as on a hyperbolic set with bound B
  ix->d = tile_dim ? tile_dim : default_tile_dim(N);
  ix->np = N - ix->d;
  int32_t st;
  try {
    st = build_index(ix);
  } catch (const std::bad_alloc &) {
    st = hs::fail(HS_E_NOMEM, "hs_index_create_total_degree: out of host memory");
  }
  if (st != HS_OK) {
    delete ix;
    return st;
  }
  *out = ix;
  return HS_OK;
}

extern "C" int32_t hs_index_create_from_list(int32_t N, int64_t n, const uint16_t *k_host, hs_index *out) {
  if (!out) return hs::fail(HS_E_INVALID, "hs_index_create_from_list: out is NULL");
  *out = nullptr;
  if (N < 1 || N > HS_NMAX) return hs::fail(HS_E_INVALID, "hs_index_create_from_list: N out of range 1..16");
  if (n < 1 || !k_host) return hs::fail(HS_E_INVALID, "hs_index_create_from_list: empty list");
  if (n >= (INT64_C(1) << 31) - 1) return hs::fail(HS_E_OVERFLOW, "hs_index_create_from_list: 2^31 or more rows");
  hs_index_s *ix = new (std::nothrow) hs_index_s();
  if (!ix) return hs::fail(HS_E_NOMEM, "hs_index_create_from_list: out of host memory");
  int32_t st = HS_OK;
  try {
    std::unique_ptr<ListSet> L(new ListSet());
    L->N = N;
    // lexicographic order of the rows
    std::vector<int64_t> order(n);
    for (int64_t r = 0; r < n; ++r) order[r] = r;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return std::lexicographical_compare(k_host + a * N, k_host + (a + 1) * N, k_host + b * N, k_host + (b + 1) * N);
    });
    L->k.resize((size_t)n * N);
    std::vector<int32_t> m(N);
    int64_t maxc = 0;
    for (int64_t r = 0; r < n && st == HS_OK; ++r) {
      for (int i = 0; i < N; ++i) {
        m[i] = k_host[order[r] * N + i];
        L->k[(size_t)r * N + i] = (uint16_t)m[i];
        maxc = std::max<int64_t>(maxc, m[i]);
      }
      if (!L->pos.emplace(ListSet::key(m.data(), N), r).second)
        st = hs::fail(HS_E_INVALID, "hs_index_create_from_list: a multi-index appears twice");
    }
    // downward closed: k - e_l is in the set whenever k_l > 0
    for (int64_t r = 0; r < n && st == HS_OK; ++r) {
      for (int i = 0; i < N; ++i) m[i] = L->k[(size_t)r * N + i];
      for (int i = 0; i < N && st == HS_OK; ++i) {
        if (m[i] == 0) continue;
        --m[i];
        if (!L->pos.count(ListSet::key(m.data(), N)))
          st = hs::fail(HS_E_INVALID, "hs_index_create_from_list: the set is not downward closed");
        ++m[i];
      }
    }
    if (st == HS_OK) {
      // N >= 3 (and N = 1): tiles are the prefixes (first N - 1 coordinates) and the
      // suffix the last coordinate, whose fibre {0..L-1} is an initial segment of the one
      // suffix list {0..maxlen-1} for every downward-closed set.  N = 2 keeps one row per
      // tile (its prefix and suffix sets would both be one-dimensional).
      L->d = (N == 2) ? 0 : 1;
      if (L->d == 1) {
        const int np = N - 1;
        for (int64_t r = 0; r < n; ++r) {
          const uint16_t *row = L->k.data() + (size_t)r * N;
          const bool fresh = r == 0 || !std::equal(row, row + np, row - N);
          if (fresh) {
            for (int i = 0; i < np; ++i) m[i] = row[i];
            L->ppos.emplace(ListSet::key(m.data(), np), (int64_t)L->flen.size());
            L->pfx.insert(L->pfx.end(), row, row + np);
            L->flen.push_back(0);
          }
          L->flen.back() += 1;
          L->maxlen = std::max(L->maxlen, L->flen.back());
        }
      }
      ix->N = N;
      ix->kind = HS_SET_LIST;
      ix->B = maxc + 1;  // coordinates stay below B
      ix->d = L->d;
      ix->np = N - L->d;
      ix->list = std::move(L);
      st = build_index(ix);
    }
  } catch (const std::bad_alloc &) {
    st = hs::fail(HS_E_NOMEM, "hs_index_create_from_list: out of host memory");
  }
  if (st != HS_OK) {
    delete ix;
    return st;
  }
  *out = ix;
  return HS_OK;
}

extern "C" int32_t hs_index_embed(hs_index sub, hs_index box, int32_t *map_host) {
  if (!sub || !box || !map_host) return hs::fail(HS_E_INVALID, "hs_index_embed: NULL argument");
  if (sub->N != box->N) return hs::fail(HS_E_INVALID, "hs_index_embed: the sets differ in N");
  const int N = sub->N, np = box->np, d = box->d;
  try {
    // row of a multi-index in the target: tile = lexicographic rank of the prefix among
    // the target's prefixes, offset = position of the suffix in the graded suffix list
    const SetOps S = set_ops(box);
    const Ranker Rp(&S, np), Rs(&S, d);
    std::vector<int64_t> off_of_lex(box->ng, -1);
    std::vector<int32_t> m(N);
    for (int64_t g = 0; g < box->ng; ++g) {
      for (int a = 0; a < d; ++a) m[a] = box->gsidx[g * d + a];
      off_of_lex[Rs.rank(m.data())] = g;
    }
    std::vector<uint16_t> k((size_t)sub->size * N);
    hs_index_multi_indices(sub, k.data());
    for (int64_t r = 0; r < sub->size; ++r) {
      for (int i = 0; i < N; ++i) m[i] = k[(size_t)r * N + i];
      if (!S.member(m.data(), N)) {
        map_host[r] = -1;
        continue;
      }
      const int64_t t = Rp.rank(m.data());
      const int64_t o = off_of_lex[Rs.rank(m.data() + np)];
      map_host[r] = (int32_t)(box->tstart[t] + o);
    }
  } catch (const std::bad_alloc &) {
    return hs::fail(HS_E_NOMEM, "hs_index_embed: out of host memory");
  }
  return HS_OK;
}

extern "C" int32_t hs_index_destroy(hs_index idx) {
  if (!idx) return HS_OK;
  if (idx->pinned) (void)hipHostFree(idx->pinned);
  delete idx;
  return HS_OK;
}

extern "C" int32_t hs_index_size(hs_index idx, int64_t *n) {
  if (!idx || !n) return hs::fail(HS_E_INVALID, "hs_index_size: NULL argument");
  *n = idx->size;
  return HS_OK;
}

extern "C" int32_t hs_index_info(hs_index idx, int32_t *tile_dim, int64_t *ntiles, int64_t *nsuffix) {
  if (!idx) return hs::fail(HS_E_INVALID, "hs_index_info: NULL handle");
  if (tile_dim) *tile_dim = idx->d;
  if (ntiles) *ntiles = idx->ntiles;
  if (nsuffix) *nsuffix = idx->ng;
  return HS_OK;
}

extern "C" int32_t hs_index_multi_indices(hs_index idx, uint16_t *out) {
  if (!idx || !out) return hs::fail(HS_E_INVALID, "hs_index_multi_indices: NULL argument");
  const int N = idx->N, d = idx->d, np = idx->np;
  for (int64_t t = 0; t < idx->ntiles; ++t)
    for (int64_t r = idx->tstart[t]; r < idx->tstart[t + 1]; ++r) {
      int64_t o = r - idx->tstart[t];
      uint16_t *dst = out + r * N;
      for (int i = 0; i < np; ++i) dst[i] = idx->tpfx[t * np + i];
      for (int a = 0; a < d; ++a) dst[np + a] = idx->gsidx[o * d + a];
    }
  return HS_OK;
}

// ---- fibres for chained recurrence passes ----------------------------------------------
// A recurrence pass along axis l couples each row with its neighbours k -+ e_l only, so a
// chain of K passes along l can run on one fibre (the rows that differ in k_l alone) at a
// time, in fast memory.  Fibres longer than kFibCore are cut into segments; each segment
// carries up to kChainMax positions of its fibre on either side as a halo, which a chain
// of at most kChainMax steps needs to get the core positions right.  Segments are packed
// whole, in the order of their fibre's first row, into batches of at most kFibBatch
// positions (see flush below for the order inside a batch).

namespace {

// row of the neighbour r + e_l, or -1
int64_t row_up(const hs_index_s *ix, int64_t r, int l) {
  const int32_t t = ix->rowtile[r];
  const int64_t o = r - ix->tstart[t];
  if (l < ix->np) {
    const int32_t u = ix->tnbr[(int64_t)t * 2 * ix->np + 2 * l + 1];
    if (u < 0 || o >= ix->tlen[u]) return -1;
    return ix->tstart[u] + o;
  }
  const int a = l - ix->np;
  const int32_t g = ix->gnbr[o * 2 * ix->d + 2 * a + 1];
  if (g < 0 || g >= ix->tlen[t]) return -1;
  return ix->tstart[t] + g;
}

int coord_of(const hs_index_s *ix, int64_t r, int l) {
  const int32_t t = ix->rowtile[r];
  if (l < ix->np) return ix->tpfx[(int64_t)t * ix->np + l];
  return ix->gsidx[(r - ix->tstart[t]) * ix->d + (l - ix->np)];
}

}  // namespace

static int32_t build_fibres(hs_index idx) {
  const int N = idx->N;
  std::vector<uint64_t> pos;
  std::vector<uint32_t> del;
  std::vector<int64_t> bat;
  std::vector<int64_t> fpos0(N), fbat0(N), fnb(N);
  std::vector<int64_t> fib;  // rows of the current fibre
  // segments of the batch being filled: (first, count) into seg_rows / seg_fl
  std::vector<std::pair<int64_t, int64_t>> segs;
  std::vector<uint64_t> seg_pos;
  for (int l = 0; l < N; ++l) {
    fpos0[l] = (int64_t)pos.size();
    fbat0[l] = (int64_t)bat.size();
    const int64_t first = (int64_t)pos.size();
    bat.push_back(0);  // batch starts relative to fpos0[l]
    // Positions of a batch: along a prefix axis in k-major order (the k-th positions of
    // all its segments, longest segment first, then the (k+1)-th ...), where neighbouring
    // fibres of one tile column sit at consecutive rows; along a suffix axis fibre after
    // fibre.  del holds each position's distance to its k - 1 and k + 1 positions.
    const bool kmajor = l < idx->np;
    auto flush = [&]() {
      if (segs.empty()) return;
      if (!kmajor) {
        for (const auto &sg : segs)
          for (int64_t t = 0; t < sg.second; ++t) {
            pos.push_back(seg_pos[(size_t)(sg.first + t)]);
            del.push_back(1u | (1u << 16));
          }
      } else {
        std::stable_sort(segs.begin(), segs.end(),
                         [](const auto &u, const auto &v) { return u.second > v.second; });
        const int64_t T = segs[0].second;
        std::vector<int64_t> cnt((size_t)T, 0);
        for (const auto &sg : segs)
          for (int64_t t = 0; t < sg.second; ++t) cnt[(size_t)t]++;
        for (int64_t t = 0; t < T; ++t)
          for (int64_t q = 0; q < cnt[(size_t)t]; ++q) {
            pos.push_back(seg_pos[(size_t)(segs[(size_t)q].first + t)]);
            const uint32_t lo = t > 0 ? (uint32_t)cnt[(size_t)t - 1] : 0u, hi = (uint32_t)cnt[(size_t)t];
            del.push_back(lo | (hi << 16));
          }
      }
      bat.push_back((int64_t)pos.size() - first);
      segs.clear();
      seg_pos.clear();
    };
    int64_t in_batch = 0;
    for (int64_t r = 0; r < idx->size; ++r) {
      if (coord_of(idx, r, l) != 0) continue;  // fibres start at k_l = 0
      fib.clear();
      for (int64_t q = r; q >= 0; q = row_up(idx, q, l)) fib.push_back(q);
      const int64_t L = (int64_t)fib.size();
      if (L > 65535) return hs::fail(HS_E_OVERFLOW, "hs_index_build_fibres: fibre longer than 65535");
      for (int64_t c0 = 0; c0 < L; c0 += hs::kFibCore) {
        const int64_t c1 = std::min<int64_t>(L, c0 + hs::kFibCore);
        const int64_t h0 = std::max<int64_t>(0, c0 - hs::kChainMax), h1 = std::min<int64_t>(L, c1 + hs::kChainMax);
        const int64_t n = h1 - h0;
        if (in_batch + n > hs::kFibBatch) {
          flush();
          in_batch = 0;
        }
        segs.emplace_back((int64_t)seg_pos.size(), n);
        for (int64_t k = h0; k < h1; ++k) {
          uint64_t fl = 0;
          if (k > h0) fl |= 1;          // k - 1 is a position of the batch
          if (k + 1 < h1) fl |= 2;      // k + 1 is a position of the batch
          if (k >= c0 && k < c1) fl |= 4;
          seg_pos.push_back((uint64_t)fib[(size_t)k] | ((uint64_t)k << 32) | (fl << 48));
        }
        in_batch += n;
      }
    }
    flush();
    fnb[l] = (int64_t)bat.size() - fbat0[l] - 1;
  }
  // append to the device image
  int64_t off = idx->dev_bytes;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off = hs::align_up(off + std::max<int64_t>(bytes, 1), 256);
    return o;
  };
  idx->off_fpos = take((int64_t)pos.size() * 8);
  idx->off_fdel = take((int64_t)del.size() * 4);
  idx->off_fbat = take((int64_t)bat.size() * 8);
  idx->blob.resize(off, 0);
  std::memcpy(idx->blob.data() + idx->off_fpos, pos.data(), pos.size() * 8);
  std::memcpy(idx->blob.data() + idx->off_fdel, del.data(), del.size() * 4);
  std::memcpy(idx->blob.data() + idx->off_fbat, bat.data(), bat.size() * 8);
  idx->dev_bytes = off;
  idx->fpos0 = fpos0;
  idx->fbat0 = fbat0;
  idx->fnb = fnb;
  idx->fibres = true;
  if (idx->pinned) {  // the staging copy no longer matches the image
    (void)hipHostFree(idx->pinned);
    idx->pinned = nullptr;
  }
  return HS_OK;
}

// the lists take 12 bytes per row and axis (plus halos); more than this is refused
static const int64_t kFibreBytesMax = int64_t(16) << 30;

extern "C" int32_t hs_index_build_fibres(hs_index idx) {
  if (!idx) return hs::fail(HS_E_INVALID, "hs_index_build_fibres: NULL handle");
  if (idx->fibres) return HS_OK;
  if (idx->size >= (int64_t)INT32_MAX)
    return hs::fail(HS_E_OVERFLOW, "hs_index_build_fibres: rows must fit 31 bits");
  if ((double)idx->size * idx->N * 12.0 * (1.0 + 16.0 / hs::kFibCore) > (double)kFibreBytesMax)
    return hs::fail(HS_E_OVERFLOW, "hs_index_build_fibres: the fibre lists would exceed 16 GiB");
  try {
    return build_fibres(idx);
  } catch (const std::bad_alloc &) {
    return hs::fail(HS_E_NOMEM, "hs_index_build_fibres: out of host memory");
  }
}

extern "C" int32_t hs_index_device_bytes(hs_index idx, int64_t *bytes) {
  if (!idx || !bytes) return hs::fail(HS_E_INVALID, "hs_index_device_bytes: NULL argument");
  *bytes = idx->dev_bytes;
  return HS_OK;
}

extern "C" int32_t hs_index_upload(hs_index idx, void *dev, int64_t bytes, void *stream) {
  if (!idx || !dev) return hs::fail(HS_E_INVALID, "hs_index_upload: NULL argument");
  if (bytes < idx->dev_bytes) return hs::fail(HS_E_WORKSPACE, "hs_index_upload: device buffer too small");
  if (reinterpret_cast<uintptr_t>(dev) % 16) return hs::fail(HS_E_INVALID, "hs_index_upload: device pointer not 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!idx->pinned) {
    HS_HIP(hipHostMalloc(&idx->pinned, idx->dev_bytes, hipHostMallocDefault));
    std::memcpy(idx->pinned, idx->blob.data(), idx->dev_bytes);
  }
  HS_HIP(hipMemcpyAsync(dev, idx->pinned, idx->dev_bytes, hipMemcpyHostToDevice, s));
  idx->fibres_uploaded = idx->fibres;
  return HS_OK;
}
