// Potential compiler: the polynomial W^pol of paper Sec. 1.3 given as terms
// prod_l p_{a_l}(x_l) in one per-axis three-term-recurrence family, with coefficients
// beta_t(t) = base_t + amp_t sin(freq_t t + phase_t).
//
// Two execution forms of the same operator W^pol(X_K) (Sec. 3.2, eq. Horner):
//  * fused: every monomial of the expanded potential is x_l^a (a <= 3) or
//    x_l^a x_{l+1} (a <= 2).  Because p(X) is linear in the polynomial p for each axis,
//    a term equals the same combination of products X_l^a X_{l+1}^b (X_{l+1} first);
//    the compiler records that combination as a matrix M (slots x terms).
//  * generic: a program of recurrence passes over whole vectors, organised as a trie
//    over the axes N..1 so that terms sharing their innermost factors share the passes.
#include <algorithm>
#include <cmath>
#include <map>
#include <new>

#include "hs_internal.h"

namespace {

// recurrence p_{k+1} = (A_k x + B_k) p_k - C_k p_{k-1}, p_0 = 1
void rec_coeffs(int basis, double scale, int k, double *A, double *Bc, double *C) {
  if (basis == HS_BASIS_MONO) {
    *A = 1.0; *Bc = 0.0; *C = 0.0;
  } else if (basis == HS_BASIS_CHEB) {  // T_a(x / L)
    *A = (k == 0 ? 1.0 : 2.0) / scale; *Bc = 0.0; *C = (k == 0 ? 0.0 : 1.0);
  } else {                              // H_a(x / s), physicists'
    *A = 2.0 / scale; *Bc = 0.0; *C = 2.0 * k;
  }
}

// monomial coefficients of p_a (index = power)
std::vector<double> mono_coeffs(int basis, double scale, int a) {
  std::vector<double> pm(a + 2, 0.0), p(a + 2, 0.0);
  p[0] = 1.0;
  for (int k = 0; k < a; ++k) {
    double A, Bc, C;
    rec_coeffs(basis, scale, k, &A, &Bc, &C);
    std::vector<double> nx(a + 2, 0.0);
    for (int i = 0; i <= a; ++i) {
      if (i + 1 <= a + 1) nx[i + 1] += A * p[i];
      nx[i] += Bc * p[i] - C * pm[i];
    }
    pm = p;
    p = nx;
  }
  p.resize(a + 1);
  return p;
}

// slot numbering of the fused form
inline int slot_a(int l, int p) { return l * 5 + (p - 1); }      // x_l^p, p = 1..3
inline int slot_g(int l, int p) { return l * 5 + 3 + (p - 1); }  // x_l^p x_{l+1}, p = 1..2
inline int slot_c(int N) { return 5 * N; }                       // constant

bool try_fused(hs_pot_s *P) {
  const int N = P->N;
  P->nslots = 5 * N + 1;
  P->M.assign((size_t)P->nslots * P->nterms, 0.0);
  for (int t = 0; t < P->nterms; ++t) {
    // expand prod_l p_{a_l}(x_l) into monomials: iterate over the product of the
    // per-axis monomial lists, skipping zero coefficients
    std::vector<std::vector<double>> mc(N);
    for (int l = 0; l < N; ++l) mc[l] = mono_coeffs(P->basis, P->scale, P->deg[t * N + l]);
    std::vector<int> pw(N, 0);
    while (true) {
      double coef = 1.0;
      for (int l = 0; l < N && coef != 0.0; ++l) coef *= mc[l][pw[l]];
      if (coef != 0.0) {
        std::vector<int> ax;
        for (int l = 0; l < N; ++l)
          if (pw[l] > 0) ax.push_back(l);
        int slot = -1;
        if (ax.empty()) {
          slot = slot_c(N);
        } else if (ax.size() == 1) {
          if (pw[ax[0]] <= 3) slot = slot_a(ax[0], pw[ax[0]]);
        } else if (ax.size() == 2 && ax[1] == ax[0] + 1 && pw[ax[1]] == 1 && pw[ax[0]] <= 2) {
          slot = slot_g(ax[0], pw[ax[0]]);
        }
        if (slot < 0) return false;
        P->M[(size_t)slot * P->nterms + t] += coef;
      }
      int l = N - 1;
      while (l >= 0) {
        if (++pw[l] < (int)mc[l].size()) break;
        pw[l] = 0;
        --l;
      }
      if (l < 0) break;
    }
  }
  // x_l^2 and x_l x_{l+1} slots: needed if some contributing term is time dependent or
  // the time-independent contributions do not cancel (the harmonic part of V cancels
  // against the subtracted |x|^2 / 2 exactly)
  P->x2 = false;
  P->x2_struct = false;
  for (int l = 0; l < N; ++l)
    for (int slot : {slot_a(l, 2), slot_g(l, 1)}) {
      double val = 0.0;
      bool dyn = false, any = false;
      for (int t = 0; t < P->nterms; ++t) {
        const double m = P->M[(size_t)slot * P->nterms + t];
        if (m == 0.0) continue;
        any = true;
        if (P->amp[t] != 0.0) dyn = true;
        val += m * P->base[t];
      }
      if (any) P->x2_struct = true;
      if (dyn || val != 0.0) P->x2 = true;
    }
  return true;
}

// ---- generic trie program ---------------------------------------------------------
struct TrieBuilder {
  hs_pot_s *P;
  int N;
  std::vector<int> order;  // term indices sorted by reversed degree vectors
  int next_slot = 2;       // slot 0: input c, slot 1: output y
  int max_slot = 2;

  int deg(int t, int l) const { return P->deg[t * N + l]; }

  // terms [lo, hi) share degrees on axes > lvl; vec holds prod_{l > lvl} p(X_l) c
  void rec(int lo, int hi, int lvl, int vec) {
    if (lvl < 0) {
      for (int i = lo; i < hi; ++i) {
        hs::PassOp op{};
        op.kind = 1;
        op.axis = -1;
        op.src = vec;
        op.prev = -1;
        op.dst = 1;
        op.term = order[i];
        P->prog.push_back(op);
      }
      return;
    }
    // three rotating slots for p_{k-1}, p_k, p_{k+1} of this axis
    const int S[3] = {next_slot, next_slot + 1, next_slot + 2};
    next_slot += 3;
    max_slot = std::max(max_slot, next_slot);
    int prev = -1, cur = vec, k = 0;
    int i = lo;
    while (i < hi) {
      const int a = deg(order[i], lvl);
      int j = i;
      while (j < hi && deg(order[j], lvl) == a) ++j;
      int last_op = -1;
      while (k < a) {
        double A, Bc, C;
        rec_coeffs(P->basis, P->scale, k, &A, &Bc, &C);
        int dst = -1;
        for (int s : S)
          if (s != prev && s != cur) {
            dst = s;
            break;
          }
        hs::PassOp op{};
        op.kind = 0;
        op.axis = lvl;
        op.src = cur;
        op.prev = (k == 0 ? -1 : prev);
        op.dst = dst;
        op.A = A;
        op.Bc = Bc;
        op.C = (k == 0 ? 0.0 : C);
        op.term = -1;
        last_op = (int)P->prog.size();
        P->prog.push_back(op);
        prev = cur;
        cur = dst;
        ++k;
      }
      if (lvl == 0 && j - i == 1 && last_op >= 0) {
        // the pass that produced this leaf also accumulates it into y
        P->prog[last_op].term = order[i];
      } else {
        rec(i, j, lvl - 1, cur);
      }
      i = j;
    }
    next_slot -= 3;
  }
};

}  // namespace

namespace hs {

int32_t compile_potential(hs_pot_s *P) {
  const int N = P->N;
  P->fused = try_fused(P);
  P->prog.clear();
  if (!P->fused) {
    // generic program: sort terms by (a_N, a_{N-1}, ..., a_1) and build the trie
    TrieBuilder tb{P, N, {}};
    tb.order.resize(P->nterms);
    for (int t = 0; t < P->nterms; ++t) tb.order[t] = t;
    std::stable_sort(tb.order.begin(), tb.order.end(), [&](int x, int y) {
      for (int l = N - 1; l >= 0; --l)
        if (P->deg[x * N + l] != P->deg[y * N + l]) return P->deg[x * N + l] < P->deg[y * N + l];
      return false;
    });
    tb.rec(0, P->nterms, N - 1, 0);
    P->nslots_vec = tb.max_slot;
  }
  // device block layout
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off = align_up(off + std::max<int64_t>(bytes, 1), 256);
    return o;
  };
  P->off_beta = take(8 * kMaxTerms);
  P->off_base = take(8 * P->nterms);
  P->off_amp = take(8 * P->nterms);
  P->off_freq = take(8 * P->nterms);
  P->off_phase = take(8 * P->nterms);
  P->off_M = take(8 * (int64_t)std::max(1, P->nslots) * P->nterms);
  P->off_hh = take(8 * (int64_t)std::max(1, P->nslots));
  P->dev_bytes = off;
  return HS_OK;
}

}  // namespace hs

extern "C" int32_t hs_pot_create(int32_t N, int32_t basis, double scale, int32_t nterms,
                                 const uint16_t *degrees, const double *base, const double *amp,
                                 const double *freq, const double *phase,
                                 int32_t subtract_harmonic, hs_pot *out) {
  if (!out) return hs::fail(HS_E_INVALID, "hs_pot_create: out is NULL");
  *out = nullptr;
  if (N < 1 || N > HS_NMAX) return hs::fail(HS_E_INVALID, "hs_pot_create: N out of range");
  if (basis < HS_BASIS_MONO || basis > HS_BASIS_HERM) return hs::fail(HS_E_INVALID, "hs_pot_create: unknown basis");
  if (!(scale > 0.0) || !std::isfinite(scale)) return hs::fail(HS_E_INVALID, "hs_pot_create: scale must be positive");
  if (nterms < 0 || (nterms > 0 && (!degrees || !base))) return hs::fail(HS_E_INVALID, "hs_pot_create: bad term arrays");
  if (subtract_harmonic && basis != HS_BASIS_MONO)
    return hs::fail(HS_E_UNSUPPORTED, "hs_pot_create: subtract_harmonic needs the monomial basis");
  const int total = nterms + (subtract_harmonic ? N : 0);
  if (total > hs::kMaxTerms) return hs::fail(HS_E_UNSUPPORTED, "hs_pot_create: more than 512 terms");
  hs_pot_s *P = new (std::nothrow) hs_pot_s();
  if (!P) return hs::fail(HS_E_NOMEM, "hs_pot_create: out of host memory");
  P->N = N;
  P->basis = basis;
  P->scale = scale;
  P->nterms = total;
  P->deg.assign((size_t)total * N, 0);
  P->base.assign(total, 0.0);
  P->amp.assign(total, 0.0);
  P->freq.assign(total, 0.0);
  P->phase.assign(total, 0.0);
  for (int t = 0; t < nterms; ++t) {
    for (int l = 0; l < N; ++l) {
      if (degrees[t * N + l] > 64) {
        delete P;
        return hs::fail(HS_E_UNSUPPORTED, "hs_pot_create: per-axis degree above 64");
      }
      P->deg[t * N + l] = degrees[t * N + l];
    }
    P->base[t] = base[t];
    P->amp[t] = amp ? amp[t] : 0.0;
    P->freq[t] = freq ? freq[t] : 0.0;
    P->phase[t] = phase ? phase[t] : 0.0;
    if (!std::isfinite(P->base[t]) || !std::isfinite(P->amp[t]) || !std::isfinite(P->freq[t]) ||
        !std::isfinite(P->phase[t])) {
      delete P;
      return hs::fail(HS_E_NONFINITE, "hs_pot_create: non-finite coefficient");
    }
  }
  for (int l = 0; l < (subtract_harmonic ? N : 0); ++l) {  // W = V - x_l^2 / 2
    P->deg[(nterms + l) * N + l] = 2;
    P->base[nterms + l] = -0.5;
  }
  int32_t st = hs::compile_potential(P);
  if (st != HS_OK) {
    delete P;
    return st;
  }
  *out = P;
  return HS_OK;
}

extern "C" int32_t hs_pot_destroy(hs_pot pot) {
  delete pot;
  return HS_OK;
}

extern "C" int32_t hs_pot_is_fused(hs_pot pot, int32_t *fused) {
  if (!pot || !fused) return hs::fail(HS_E_INVALID, "hs_pot_is_fused: NULL argument");
  *fused = pot->fused ? 1 : 0;
  return HS_OK;
}

extern "C" int32_t hs_pot_device_bytes(hs_pot pot, int64_t *bytes) {
  if (!pot || !bytes) return hs::fail(HS_E_INVALID, "hs_pot_device_bytes: NULL argument");
  *bytes = pot->dev_bytes;
  return HS_OK;
}
