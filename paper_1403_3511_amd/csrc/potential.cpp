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
  // the time-dependent terms reach only the linear and constant slots (a laser-type
  // drive): the difference of two coefficient sets is then linear in the coordinates
  P->dyn_linear = true;
  for (int slot = 0; slot < P->nslots; ++slot) {
    if (slot == slot_c(N) || slot % 5 == 0) continue;  // x_l^1 and the constant
    for (int t = 0; t < P->nterms; ++t)
      if (P->amp[t] != 0.0 && P->M[(size_t)slot * P->nterms + t] != 0.0) P->dyn_linear = false;
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
        op.plus = -1;
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
        op.plus = -1;
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

// ---- split program: trie over the inner axes, Clenshaw sums over the outer axes ----
// With outer axes 0..s-1 and inner axes s..N-1 (axis N-1 is applied first),
//   W^pol c = sum_o p_{o_0}(X_0) ... p_{o_{s-1}}(X_{s-1}) W_o,
//   W_o = sum_{terms t with outer part o} beta_t V_{inner(t)},
//   V_i = p_{i_s}(X_s) ... p_{i_{N-1}}(X_{N-1}) c.
// The V_i come from a trie of recurrence passes (shared from c outwards), the nested
// sums over the outer axes from Clenshaw's recurrence with vector coefficients
//   b_k = u_k + (A_k X + B_k) b_{k+1} - C_{k+1} b_{k+2},  sum_k p_k(X) u_k = b_0,
// (shared from the outside inwards), and a per-row combination links the two.  Same
// operator as the trie, in exact arithmetic.
struct SplitBuilder {
  hs_pot_s *P;
  int N, s;
  std::vector<hs::PassOp> prog;
  int next = 2, max_slot = 2;
  std::vector<int> freel;
  // inner: vector slot of each inner multi-degree prefix (axes N-1 .. l), keyed by the
  // degree string of axes l..N-1
  std::map<std::vector<int>, int> inner_slot;
  std::vector<int> cin_slot, cout_slot, cptr, cidx, cterm;
  bool ok = true;

  int alloc() {
    if (!freel.empty()) {
      const int x = freel.back();
      freel.pop_back();
      return x;
    }
    const int x = next++;
    max_slot = std::max(max_slot, next);
    return x;
  }
  void release(int x) {
    if (x >= 2) freel.push_back(x);
  }
  int deg(int t, int l) const { return P->deg[t * N + l]; }
  std::vector<int> inner_key(int t, int l) const {  // degrees of axes l..N-1
    std::vector<int> k;
    for (int a = l; a < N; ++a) k.push_back(deg(t, a));
    return k;
  }
  hs::PassOp pass(int axis, int src, int prev, int dst, double A, double Bc, double C, int plus) const {
    hs::PassOp op{};
    op.kind = 0;
    op.axis = axis;
    op.src = src;
    op.prev = prev;
    op.dst = dst;
    op.A = A;
    op.Bc = Bc;
    op.C = C;
    op.term = -1;
    op.plus = plus;
    return op;
  }

  // V vectors of every inner node, level by level from axis N-1 down to axis s
  void build_inner() {
    inner_slot[std::vector<int>()] = 0;  // the input vector
    for (int l = N - 1; l >= s; --l) {
      // chains: parent key (axes l+1..N-1) -> largest degree on axis l among terms
      std::map<std::vector<int>, int> kmax;
      for (int t = 0; t < P->nterms; ++t) {
        const std::vector<int> par = inner_key(t, l + 1);
        int &m = kmax[par];
        m = std::max(m, deg(t, l));
      }
      for (const auto &kv : kmax) {
        const int u = inner_slot.at(kv.first);
        int pm = -1, pc = u;
        std::vector<int> key = kv.first;
        key.insert(key.begin(), 0);
        inner_slot[key] = u;  // p_0(X) u = u
        for (int k = 0; k < kv.second; ++k) {
          double A, Bc, C;
          rec_coeffs(P->basis, P->scale, k, &A, &Bc, &C);
          const int d = alloc();
          prog.push_back(pass(l, pc, k == 0 ? -1 : pm, d, A, Bc, k == 0 ? 0.0 : C, -1));
          key[0] = k + 1;
          inner_slot[key] = d;
          pm = pc;
          pc = d;
        }
      }
    }
  }

  // W_o for every outer multi-degree, one combination step
  std::map<std::vector<int>, int> outer_slot;
  void build_combination() {
    std::map<std::vector<int>, std::vector<std::pair<int, int>>> rows;  // outer -> (V slot, term)
    for (int t = 0; t < P->nterms; ++t) {
      std::vector<int> o;
      for (int a = 0; a < s; ++a) o.push_back(deg(t, a));
      rows[o].push_back({inner_slot.at(inner_key(t, s)), t});
    }
    std::map<int, int> in_index;
    for (auto &kv : rows)
      for (auto &e : kv.second)
        if (!in_index.count(e.first)) {
          in_index[e.first] = (int)cin_slot.size();
          cin_slot.push_back(e.first);
        }
    if ((int)cin_slot.size() > hs::kMaxComb || (int)rows.size() > hs::kMaxComb) {
      ok = false;
      return;
    }
    cptr.push_back(0);
    for (auto &kv : rows) {
      const int d = alloc();
      outer_slot[kv.first] = d;
      cout_slot.push_back(d);
      for (auto &e : kv.second) {
        cidx.push_back(in_index[e.first]);
        cterm.push_back(e.second);
      }
      cptr.push_back((int)cidx.size());
    }
    hs::PassOp op{};
    op.kind = 2;
    op.src = op.prev = op.dst = op.plus = -1;
    op.term = -1;
    prog.push_back(op);
    // inner vectors are dead after the combination (the input vector is slot 0)
    std::vector<int> dead;
    for (auto &kv : inner_slot) dead.push_back(kv.second);
    std::sort(dead.begin(), dead.end());
    dead.erase(std::unique(dead.begin(), dead.end()), dead.end());
    for (int x : dead) release(x);
  }

  // slot of sum_{o_l..o_{s-1}} p(X_l) .. p(X_{s-1}) W_{prefix, o_l..}; at l = 0 the result
  // is accumulated into y
  int build_outer(int l, const std::vector<int> &prefix) {
    if (l == s) return outer_slot.at(prefix);
    std::map<int, int> child;  // degree on axis l -> slot
    for (const auto &kv : outer_slot) {
      if (!std::equal(prefix.begin(), prefix.end(), kv.first.begin())) continue;
      const int k = kv.first[l];
      if (child.count(k)) continue;
      std::vector<int> pre = prefix;
      pre.push_back(k);
      child[k] = build_outer(l + 1, pre);
    }
    const int K = child.rbegin()->first;
    auto u = [&](int k) { return child.count(k) ? child[k] : -1; };
    if (K == 0) {
      const int r = child[0];
      if (l == 0) {
        hs::PassOp op{};
        op.kind = 1;
        op.src = r;
        op.prev = op.dst = op.plus = -1;
        op.term = hs::kTermOne;
        prog.push_back(op);
      }
      return r;
    }
    int b2 = -1, b1 = child[K];  // b_{k+2}, b_{k+1}
    bool b2_temp = false, b1_temp = false;
    for (int k = K - 1; k >= 0; --k) {
      double A, Bc, C, A1, B1, C1;
      rec_coeffs(P->basis, P->scale, k, &A, &Bc, &C);
      rec_coeffs(P->basis, P->scale, k + 1, &A1, &B1, &C1);
      const int d = alloc();
      hs::PassOp op = pass(l, b1, b2, d, A, Bc, b2 >= 0 ? C1 : 0.0, u(k));
      if (l == 0 && k == 0) op.term = hs::kTermOne;
      prog.push_back(op);
      if (b2 >= 0 && b2_temp) release(b2);
      b2 = b1;
      b2_temp = b1_temp;
      b1 = d;
      b1_temp = true;
    }
    if (b2 >= 0 && b2_temp) release(b2);
    for (auto &kv : child) release(kv.second);  // coefficient vectors consumed
    return b1;
  }

  bool build() {
    build_inner();
    build_combination();
    if (!ok) return false;
    build_outer(0, {});
    return true;
  }
};

// memory traffic of a program in vector passes (a recurrence pass reads src and its
// neighbours, prev, plus and writes dst; an accumulation reads and writes y)
double program_cost(const std::vector<hs::PassOp> &prog, int ncomb_in, int ncomb_out) {
  double c = 0.0;
  for (const auto &op : prog) {
    if (op.kind == 0) c += 2.0 + (op.prev >= 0) + (op.plus >= 0) + (op.term != -1 ? 2.0 : 0.0);
    else if (op.kind == 1) c += 3.0;
    else c += ncomb_in + ncomb_out;
  }
  return c;
}

// Chains of recurrence passes (paper Sec. 3.2: the three-term recurrence of the basis,
// applied along one axis at a time).  Op i + 1 continues op i when both are passes along
// the same axis, op i + 1 reads op i's output as its source and op i's source as its
// previous vector.  A chain runs as one launch over the fibres of its axis, so its inputs
// (first source and previous vector, the added vectors) must not be among the slots it
// writes, nor y when it accumulates into y.  An output is kept (written) when an op after
// the chain reads it before it is written again and no later step of the chain writes
// the same slot.
void analyse_chains(hs_pot_s *P) {
  const std::vector<hs::PassOp> &pg = P->prog;
  const int n = (int)pg.size();
  P->chain.assign(n, 1);
  P->keep.assign(n, 1);
  auto reads = [&](const hs::PassOp &op, int slot) {
    if (op.kind == 0) return op.src == slot || op.prev == slot || op.plus == slot || (op.term != -1 && slot == 1);
    if (op.kind == 1) return op.src == slot || slot == 1;
    for (int c : P->cin_slot) if (c == slot) return true;
    return false;
  };
  auto writes = [&](const hs::PassOp &op, int slot) {
    if (op.kind == 0) return op.dst == slot || (op.term != -1 && slot == 1);
    if (op.kind == 1) return slot == 1;
    for (int c : P->cout_slot) if (c == slot) return true;
    return false;
  };
  auto live_after = [&](int e, int slot) {
    if (slot == 0 || slot == 1) return true;
    for (int m = e; m < n; ++m) {
      if (reads(pg[m], slot)) return true;
      if (writes(pg[m], slot)) return false;
    }
    return false;
  };
  auto ok = [&](int i, int e) {
    std::vector<int> in{pg[i].src};
    if (pg[i].prev >= 0) in.push_back(pg[i].prev);
    bool term = false;
    for (int j = i; j < e; ++j) {
      if (pg[j].plus >= 0) in.push_back(pg[j].plus);
      term |= pg[j].term != -1;
    }
    for (int j = i; j < e; ++j)
      for (int v : in)
        if (pg[j].dst == v || (term && v == 1)) return false;
    return true;
  };
  int i = 0;
  while (i < n) {
    int e = i + 1;
    if (pg[i].kind == 0)
      while (e < n && e - i < hs::kChainMax && pg[e].kind == 0 && pg[e].axis == pg[i].axis &&
             pg[e].src == pg[e - 1].dst && pg[e].prev == pg[e - 1].src)
        ++e;
    while (e > i + 1 && !ok(i, e)) --e;
    if (e - i >= 2) {
      P->chain[i] = e - i;
      for (int j = i; j < e; ++j) {
        if (j > i) P->chain[j] = 0;
        bool later = false;
        for (int q = j + 1; q < e; ++q) later |= pg[q].dst == pg[j].dst;
        P->keep[j] = !later && live_after(e, pg[j].dst);
      }
    }
    i = e;
  }
}

// The split program's combination and the chains right after it along one axis (the
// Clenshaw sums of the first outer axis) can run as one launch per fibre batch: each
// position holds the combination's inputs and forms every combination output the chains
// add on the spot, so the combination outputs never pass through memory.  That needs, in
// the program's order:
//  - every chain input that is a combination output still holds that output when read
//    (no earlier chain of the group wrote its slot); other inputs are slots no chain of
//    the group writes;
//  - the slots the group writes are none of the combination's inputs and none of the
//    group's inputs read from memory (such an output is moved to a new slot first, with
//    the reads that follow renamed);
//  - combination outputs read after the group, still holding their value, are written.
// Returns the number of outputs moved to new slots (analyse_chains must run again then),
// or -1 when the group does not qualify.
int comb_group(hs_pot_s *P, bool rename) {
  std::vector<hs::PassOp> &pg = P->prog;
  const int n = (int)pg.size();
  P->cg_op = P->cg_end = -1;
  P->cg_wt.clear();
  int c = -1;
  for (int i = 0; i < n; ++i)
    if (pg[i].kind == 2) {
      c = i;
      break;
    }
  if (c < 0 || (int)P->cin_slot.size() > hs::kCombRegs || (int)P->cout_slot.size() > hs::kMaxComb) return -1;
  for (int s : P->cin_slot) {
    if (s == 1) return -1;
    // an output written through over an input would race with other workgroups' reads
    for (int o : P->cout_slot)
      if (o == s) return -1;
  }
  for (int i = c + 1; i < n; ++i)
    if (pg[i].kind == 2) return -1;  // one combination per program
  if (c + 1 >= n || pg[c + 1].kind != 0 || P->chain[c + 1] < 1) return -1;
  const int axis = pg[c + 1].axis;
  int e = c + 1, nch = 0;
  while (e < n && pg[e].kind == 0 && pg[e].axis == axis && P->chain[e] >= 1 && nch < hs::kCombChains) {
    e += P->chain[e];
    ++nch;
  }
  std::map<int, int> comb_out;  // slot -> combination output index
  for (int o = 0; o < (int)P->cout_slot.size(); ++o) comb_out[P->cout_slot[o]] = o;
  // 0: unchanged since the combination, 1: written by the group
  std::map<int, int> state;
  std::vector<int> mem_reads;
  auto read = [&](int slot) {
    if (slot < 0) return true;
    if (state.count(slot) && state[slot] == 1) return false;
    if (!comb_out.count(slot)) mem_reads.push_back(slot);
    return true;
  };
  bool term = false;
  for (int j = c + 1; j < e;) {
    const int K = P->chain[j];
    if (!read(pg[j].src) || !read(pg[j].prev)) return -1;
    for (int q = j; q < j + K; ++q) {
      if (!read(pg[q].plus)) return -1;
      term |= pg[q].term != -1;
    }
    for (int q = j; q < j + K; ++q) state[pg[q].dst] = 1;
    j += K;
  }
  if ((int)mem_reads.size() > hs::kCombChains) return -1;
  for (int v : mem_reads)
    if ((state.count(v) && state[v] == 1) || (term && v == 1)) return -1;
  // written outputs (kept) that the combination or the group's memory reads use
  std::vector<int> moved;
  for (int j = c + 1; j < e; ++j) {
    if (!P->keep[j]) continue;
    const int d = pg[j].dst;
    bool clash = false;
    for (int v : P->cin_slot) clash |= v == d;
    for (int v : mem_reads) clash |= v == d;
    if (clash) moved.push_back(j);
  }
  if (!moved.empty()) {
    if (!rename) return -1;
    for (int j : moved) {
      const int old = pg[j].dst, fresh = P->nslots_vec++;
      pg[j].dst = fresh;
      for (int m = j + 1; m < n; ++m) {
        hs::PassOp &op = pg[m];
        if (op.kind == 0) {
          if (op.src == old) op.src = fresh;
          if (op.prev == old) op.prev = fresh;
          if (op.plus == old) op.plus = fresh;
          if (op.dst == old) break;
        } else if (op.kind == 1) {
          if (op.src == old) op.src = fresh;
        } else {
          return -1;  // a second combination: not expected after the first
        }
      }
    }
    return (int)moved.size();
  }
  // combination outputs read after the group while they still hold their value
  for (const auto &kv : comb_out) {
    const int slot = kv.first;
    if (state.count(slot) && state[slot] == 1) continue;
    bool used = false;
    for (int m = e; m < n && !used; ++m) {
      const hs::PassOp &op = pg[m];
      if (op.kind == 0) {
        used = op.src == slot || op.prev == slot || op.plus == slot;
        if (op.dst == slot) break;
      } else if (op.kind == 1) {
        used = op.src == slot;
      } else {
        used = true;
      }
    }
    if (used) P->cg_wt.push_back(kv.second);
  }
  P->cg_op = c;
  P->cg_end = e;
  return 0;
}

// Consecutive chains along one axis (outside the combination's group) that read only
// memory no chain of the group writes, and whose kept outputs are none of the group's
// inputs, run as one launch over the axis's fibre batches, chain after chain.
void multi_chain_groups(hs_pot_s *P) {
  const std::vector<hs::PassOp> &pg = P->prog;
  const int n = (int)pg.size();
  P->mc_end.assign(n, 0);
  int i = 0;
  while (i < n) {
    if (pg[i].kind != 0 || P->chain[i] < 1 || (P->cg_op >= 0 && i > P->cg_op && i < P->cg_end)) {
      ++i;
      continue;
    }
    // extend while the next chain is on the same axis and independent of the group so far
    std::vector<int> in, out;
    bool term = false;
    int e = i, nch = 0;
    while (e < n && pg[e].kind == 0 && P->chain[e] >= 1 && pg[e].axis == pg[i].axis && nch < hs::kCombChains &&
           !(P->cg_op >= 0 && e > P->cg_op && e < P->cg_end)) {
      const int K = P->chain[e];
      std::vector<int> cin{pg[e].src};
      if (pg[e].prev >= 0) cin.push_back(pg[e].prev);
      bool t = false;
      for (int q = e; q < e + K; ++q) {
        if (pg[q].plus >= 0) cin.push_back(pg[q].plus);
        t |= pg[q].term != -1;
      }
      std::vector<int> cdst;
      for (int q = e; q < e + K; ++q) cdst.push_back(pg[q].dst);
      // inputs of the new chain: not written by the group so far (any step, kept or not);
      // its writes: none of the group's inputs, its own included
      bool ok = true;
      std::vector<int> all_in = in;
      all_in.insert(all_in.end(), cin.begin(), cin.end());
      for (int v : cin)
        for (int d : out) ok &= v != d;
      for (int d : cdst)
        for (int v : all_in) ok &= v != d;
      if ((t || term) && std::find(all_in.begin(), all_in.end(), 1) != all_in.end()) ok = false;
      std::vector<int> uniq = all_in;
      std::sort(uniq.begin(), uniq.end());
      uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
      if ((int)uniq.size() > hs::kCombChains) ok = false;
      if (!ok) break;
      in = all_in;
      out.insert(out.end(), cdst.begin(), cdst.end());
      term |= t;
      e += K;
      ++nch;
    }
    if (nch >= 2) {
      P->mc_end[i] = e;
      i = e;
    } else {
      i += std::max(1, P->chain[i]);
    }
  }
}

}  // namespace

namespace hs {

int32_t compile_potential(hs_pot_s *P) {
  const int N = P->N;
  P->fused = try_fused(P);
  P->prog.clear();
  P->split = 0;
  P->cin_slot.clear();
  P->cout_slot.clear();
  P->cptr.clear();
  P->cidx.clear();
  P->cterm.clear();
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
    // a split between Clenshaw sums (outer axes) and the trie (inner axes) when it moves
    // fewer vectors; slot count bounded so the workspace stays moderate
    double best = program_cost(P->prog, 0, 0);
    for (int s = 1; s <= N && P->nterms > 0; ++s) {
      SplitBuilder sb{P, N, s};
      if (!sb.build() || sb.max_slot > 160) continue;
      const double c = program_cost(sb.prog, (int)sb.cin_slot.size(), (int)sb.cout_slot.size());
      if (c < 0.8 * best) {
        best = c;
        P->split = s;
        P->prog = sb.prog;
        P->nslots_vec = sb.max_slot;
        P->cin_slot = sb.cin_slot;
        P->cout_slot = sb.cout_slot;
        P->cptr = sb.cptr;
        P->cidx = sb.cidx;
        P->cterm = sb.cterm;
      }
    }
  }
  analyse_chains(P);
  if (!P->fused && comb_group(P, true) > 0) {
    analyse_chains(P);
    comb_group(P, false);
  }
  multi_chain_groups(P);
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
  P->off_comb = take(4 * (int64_t)(P->cptr.size() + 2 * P->cidx.size()));  // cptr | cidx | cterm
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
