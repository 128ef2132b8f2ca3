/* Compiled CPU oracle of the fast algorithm (O-fast), plain C with OpenMP loops.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/ and by the CPU-baseline leg of bench.py, never
 * by the product library, and it shares no code with it.  It restates the same passages
 * as oracle/operators.py, in the same order, for sets too large for NumPy:
 *
 *   - the index set K = { k in N_0^N : prod_l (1 + k_l) <= B } in lexicographic order,
 *     k_N fastest (Sec. 1.2, definition of the hyperbolically reduced set);
 *   - the direct operation (X^(l) v)_j = sqrt(j_l / 2) v_{j - e_l}
 *     + sqrt((j_l + 1) / 2) v_{j + e_l}, a neighbour outside K contributing nothing
 *     (Sec. 3.1, eq. DirectOperationWithX);
 *   - formal insertion W^pol(X_K) v = sum_t beta_t prod_l p_{a_{t,l}}(X^(l)) v, each term
 *     started again from v, axis N applied first (Sec. 3.2, eq. Horner; Fig. 3), with
 *     p_a by its three-term recurrence p_{k+1} = (A_k x + B_k) p_k - C_k p_{k-1};
 *   - the diagonal D_jj = sum_l (j_l + 1/2) (Sec. 1.1).
 *
 * Neighbours are found by ranking k +- e_l in the lexicographic enumeration:
 *   rank(k) = sum_l sum_{a < k_l} |K_{N-l}(floor(B_l / (1 + a)))|,  B_1 = B,
 *   B_{l+1} = floor(B_l / (1 + k_l)),
 * with the inner sums tabulated per level and per distinct remaining bound.
 * Every loop over rows is an OpenMP loop; each row is computed independently, so the
 * result does not depend on the number of threads.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct fc_set {
  int N;
  int64_t B, n;
  uint16_t *k;      /* n x N multi-indices, lexicographic */
  int64_t *nbr;     /* [2N][n]: 2l -> rank of k - e_l, 2l+1 -> rank of k + e_l, -1 if absent */
} fc_set;

/* |K_m(b)| for m <= N, b <= B: cnt[m][b], by the divisor-sum recursion
 * |K_m(b)| = sum_{a=1..b} |K_{m-1}(floor(b / a))|, |K_0(b)| = 1 for b >= 1. */
static int64_t **count_table(int N, int64_t B) {
  int64_t **cnt = (int64_t **)malloc(sizeof(int64_t *) * (N + 1));
  for (int m = 0; m <= N; ++m) {
    cnt[m] = (int64_t *)calloc((size_t)B + 1, sizeof(int64_t));
    for (int64_t b = 1; b <= B; ++b) {
      if (m == 0) {
        cnt[m][b] = 1;
        continue;
      }
      int64_t s = 0;
      for (int64_t a = 1; a <= b; ++a) s += cnt[m - 1][b / a];
      cnt[m][b] = s;
    }
  }
  return cnt;
}

/* cum[l][b][a] = sum_{a' < a} |K_{N-1-l}(floor(b / (1 + a')))| for every b that occurs
 * as a remaining bound (b = floor(B / q)), stored flat with per-b offsets. */
typedef struct {
  int64_t *off;  /* [B + 1] start of b's run in cum, or -1 */
  int64_t *cum;
} level_table;

static level_table *rank_tables(int N, int64_t B, int64_t **cnt) {
  level_table *T = (level_table *)malloc(sizeof(level_table) * N);
  for (int l = 0; l < N; ++l) {
    const int rest = N - 1 - l;
    T[l].off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)B + 1));
    for (int64_t b = 0; b <= B; ++b) T[l].off[b] = -1;
    int64_t total = 0;
    for (int64_t b = 1; b <= B; ++b)
      if (B / (B / b) == b) total += b + 1; /* b = floor(B / q) for some q */
    T[l].cum = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    int64_t pos = 0;
    for (int64_t b = 1; b <= B; ++b) {
      if (B / (B / b) != b) continue;
      T[l].off[b] = pos;
      int64_t s = 0;
      T[l].cum[pos] = 0;
      for (int64_t a = 0; a < b; ++a) {
        s += cnt[rest][b / (1 + a)];
        T[l].cum[pos + a + 1] = s;
      }
      pos += b + 1;
    }
  }
  return T;
}

/* rank of the multi-index k (given as ints), or -1 if it is not in K */
static int64_t rank_of(int N, int64_t B, const level_table *T, const int *k) {
  int64_t b = B, r = 0;
  for (int l = 0; l < N; ++l) {
    if (k[l] < 0 || k[l] >= b) return -1;
    r += T[l].cum[T[l].off[b] + k[l]];
    b = b / (1 + k[l]);
  }
  return r;
}

fc_set *fc_set_create(int N, int64_t B) {
  if (N < 1 || N > 16 || B < 1 || B > 16384) return NULL;
  int64_t **cnt = count_table(N, B);
  fc_set *S = (fc_set *)calloc(1, sizeof(fc_set));
  S->N = N;
  S->B = B;
  S->n = cnt[N][B];
  S->k = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)S->n * N);
  /* lexicographic enumeration: odometer over k with the product rule */
  {
    int k[16] = {0};
    int64_t bnd[17];
    bnd[0] = B;
    for (int l = 0; l < N; ++l) bnd[l + 1] = bnd[l];
    for (int64_t r = 0; r < S->n; ++r) {
      for (int l = 0; l < N; ++l) S->k[r * N + l] = (uint16_t)k[l];
      /* next: increment the last axis that can grow, reset the ones after it */
      int l = N - 1;
      while (l >= 0) {
        if (k[l] + 1 < bnd[l]) break; /* (1 + k_l + 1) <= bnd_l  <=>  k_l + 1 < bnd_l */
        --l;
      }
      if (l < 0) break;
      k[l] += 1;
      bnd[l + 1] = bnd[l] / (1 + k[l]);
      for (int q = l + 1; q < N; ++q) {
        k[q] = 0;
        bnd[q + 1] = bnd[q];
      }
    }
  }
  level_table *T = rank_tables(N, B, cnt);
  S->nbr = (int64_t *)malloc(sizeof(int64_t) * (size_t)S->n * 2 * N);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < S->n; ++r) {
    int k[16];
    for (int l = 0; l < N; ++l) k[l] = S->k[r * N + l];
    for (int l = 0; l < N; ++l) {
      k[l] -= 1;
      S->nbr[(int64_t)(2 * l) * S->n + r] = rank_of(N, B, T, k);
      k[l] += 2;
      S->nbr[(int64_t)(2 * l + 1) * S->n + r] = rank_of(N, B, T, k);
      k[l] -= 1;
    }
  }
  for (int l = 0; l < N; ++l) {
    free(T[l].off);
    free(T[l].cum);
  }
  free(T);
  for (int m = 0; m <= N; ++m) free(cnt[m]);
  free(cnt);
  return S;
}

int64_t fc_set_size(const fc_set *S) { return S ? S->n : -1; }

void fc_set_multi_indices(const fc_set *S, uint16_t *out) {
  memcpy(out, S->k, sizeof(uint16_t) * (size_t)S->n * S->N);
}

void fc_set_destroy(fc_set *S) {
  if (!S) return;
  free(S->k);
  free(S->nbr);
  free(S);
}

/* (A_k, B_k, C_k) of p_{k+1} = (A_k x + B_k) p_k - C_k p_{k-1}, p_0 = 1.
 * basis 0: monomials; 1: Chebyshev T_a(x / s); 2: physicists' Hermite H_a(x / s). */
static void recurrence(int basis, double s, int k, double *A, double *Bc, double *C) {
  *Bc = 0.0;
  if (basis == 0) {
    *A = 1.0;
    *C = 0.0;
  } else if (basis == 1) {
    *A = (k == 0 ? 1.0 : 2.0) / s;
    *C = k == 0 ? 0.0 : 1.0;
  } else {
    *A = 2.0 / s;
    *C = 2.0 * k;
  }
}

/* out = A X^(l) v + Bc v - C w (w may be NULL when C = 0) */
static void axis_step(const fc_set *S, int l, double A, double Bc, double C, const cplx *v, const cplx *w,
                      cplx *out) {
  const int N = S->N;
  const int64_t n = S->n;
  const int64_t *m = S->nbr + (int64_t)(2 * l) * n, *p = S->nbr + (int64_t)(2 * l + 1) * n;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    const double jl = (double)S->k[r * N + l];
    cplx x = 0.0;
    if (m[r] >= 0) x += sqrt(jl / 2.0) * v[m[r]];
    if (p[r] >= 0) x += sqrt((jl + 1.0) / 2.0) * v[p[r]];
    cplx o = A * x + Bc * v[r];
    if (C != 0.0) o -= C * w[r];
    out[r] = o;
  }
}

/* y = (D + W^pol(X_K)) v.  deg: nterms x N degrees, coef: nterms coefficients.
 * nthreads > 0 sets the OpenMP thread count.  Returns 0, or -1 on bad arguments. */
int fc_apply_h(const fc_set *S, int basis, double scale, int nterms, const uint16_t *deg, const double *coef,
               const cplx *v, cplx *y, int nthreads) {
  if (!S || !v || !y || nterms < 0 || basis < 0 || basis > 2) return -1;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  const int N = S->N;
  const int64_t n = S->n;
  cplx *u = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  cplx *wm = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  cplx *wp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  cplx *nx = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  /* the diagonal first */
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    double d = 0.5 * N;
    for (int l = 0; l < N; ++l) d += (double)S->k[r * N + l];
    y[r] = d * v[r];
  }
  for (int t = 0; t < nterms; ++t) {
    /* each term restarts from v */
    memcpy(u, v, sizeof(cplx) * (size_t)n);
    for (int l = N - 1; l >= 0; --l) {
      const int a = deg[t * N + l];
      if (a == 0) continue;
      double A, Bc, C;
      /* p_a(X^(l)) u: w_- = u, w_+ = A_0 X u + B_0 u, then the recurrence */
      memcpy(wm, u, sizeof(cplx) * (size_t)n);
      recurrence(basis, scale, 0, &A, &Bc, &C);
      axis_step(S, l, A, Bc, 0.0, wm, NULL, wp);
      for (int k = 1; k < a; ++k) {
        recurrence(basis, scale, k, &A, &Bc, &C);
        axis_step(S, l, A, Bc, C, wp, wm, nx);
        cplx *tmp = wm;
        wm = wp;
        wp = nx;
        nx = tmp;
      }
      memcpy(u, wp, sizeof(cplx) * (size_t)n);
    }
    const double c = coef[t];
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) y[r] += c * u[r];
  }
  free(u);
  free(wm);
  free(wp);
  free(nx);
  return 0;
}

int fc_max_threads(void) { return omp_get_max_threads(); }
