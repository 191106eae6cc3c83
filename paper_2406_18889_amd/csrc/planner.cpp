// Contraction planning: tree search, slicing and index layout.
//
// * Trees (Methods C): randomized greedy pairwise merging and recursive
//   min-cut bisection, then simulated annealing over local tree rotations,
//   all scored by the summed predicted time of every step over all slices.
// * Slicing (Methods C, slicing identity): wires are fixed one at a time,
//   each time the one whose slicing gives the lowest total cost, until every
//   intermediate of a slice fits the cap of 2^M elements (Methods D, the
//   target contraction treewidth M).  A subtree whose leaves touch no sliced
//   wire is the same in every slice and is computed once.
// * Closed output legs (Methods C, computing only the entries the sampled
//   strings need): a subtree holding q closed legs stores them as plain legs
//   while q < nb and as the batch index b (2^nb strings) once q >= nb; a
//   step whose result reaches q >= nb is a product batched over b whose
//   operands are gathered per string.
// * Layout (Methods C, dimension order): from the root down, each operand
//   stores [batch or gathered legs, free indices in the order of the result,
//   contracted indices last in one shared order], so both operands are read
//   as row-major matrices with the contracted coordinate fastest and no
//   permutation is materialised; the result is written through per-bit
//   strides into the layout its consumer chose.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <limits>
#include <numeric>
#include <random>
#include <stdexcept>
#include <string>
#include <thread>

#include "plan.h"

namespace lf {

namespace {

struct FlopMem : CostFn {
  // Peak rates of one MI355X: 157.3 TFLOP/s fp32 matrix, 2.5 PFLOP/s fp16
  // matrix, 8 TB/s HBM; 8 real flops per complex multiply-add; a fixed
  // launch cost per step.
  double step(int nz, int nm, int nn, int nk, int dtype) const override {
    double macs = std::ldexp(1.0, nz + nm + nn + nk);
    double es = dtype ? 4.0 : 8.0;
    double bytes = es * (std::ldexp(1.0, nz + nm + nk) + std::ldexp(1.0, nz + nn + nk) +
                         std::ldexp(1.0, nz + nm + nn));
    double peak = dtype ? 2.5e15 : 157.3e12;
    return 8.0 * macs / peak + bytes / 8.0e12 + 3.0e-6;
  }
};

struct Shape {
  int wz = 0, wm = 0, wn = 0, wk = 0;
  bool batched = false;
};

struct Ctx {
  const Network& net;
  int nidx, nb;
  Bits keep;     // open, closed (never contracted)
  Bits closed;
  std::vector<int> bits_of;
  explicit Ctx(const Network& n)
      : net(n), nidx(int(n.indices.size())), nb(n.nb), keep(nidx), closed(nidx) {
    bits_of.resize(nidx);
    for (int i = 0; i < nidx; ++i) {
      bits_of[i] = n.indices[i].bits;
      if (n.indices[i].kind != IDX_WIRE) keep.set(i);
      if (n.indices[i].kind == IDX_CLOSED) closed.set(i);
    }
  }
  // every index of a node set is one bit (wires, open and closed legs)
  int plain_bits(const Bits& b) const { return b.andnot(closed).count(); }
  int n_closed(const Bits& b) const { return (b & closed).count(); }
  bool batched(int q) const { return q > 0 && q >= nb; }
  int eff_closed(int q) const { return batched(q) ? nb : q; }
  // log2 elements of a (sliced) node
  int weight(const Bits& b) const { return plain_bits(b) + eff_closed(n_closed(b)); }
  Bits merged(const Bits& a, const Bits& b) const {
    Bits common = a & b;
    Bits gone = common.andnot(keep);
    return (a | b).andnot(gone);
  }
  Shape classify(const Bits& As, const Bits& Bs) const {
    Shape s;
    Bits common = As & Bs;
    s.wk = plain_bits(common);
    int qa = n_closed(As), qb = n_closed(Bs);
    s.batched = batched(qa + qb);
    if (s.batched) {
      s.wz = nb;
      s.wm = plain_bits(As) - s.wk;
      s.wn = plain_bits(Bs) - s.wk;
    } else {
      s.wm = plain_bits(As) + qa - s.wk;
      s.wn = plain_bits(Bs) + qb - s.wk;
    }
    if (s.wm < s.wn) std::swap(s.wm, s.wn);
    return s;
  }
};

// ----------------------------------------------------------------- greedy
// Repeatedly merge the pair of tensors sharing a wire whose score
// size(C) - alpha (size(A) + size(B)) is lowest, with Gumbel noise of the
// given temperature on the log score.  Sliced wires are removed first.  In
// the score a subtree's closed legs count at most `b_weight` bits, so trees
// that gather the sampled strings late are reachable.
void greedy_tree(const Ctx& C, const std::vector<Bits>& leaf_idx, const Bits& sliced,
                 std::mt19937_64& rng, double temperature, double alpha, int b_weight,
                 Tree& tree) {
  int L = int(leaf_idx.size());
  tree = Tree();
  tree.n_leaves = L;
  std::vector<Bits> idx(L);
  for (int i = 0; i < L; ++i) idx[i] = leaf_idx[i].andnot(sliced);
  auto hw = [&](const Bits& b) { return C.plain_bits(b) + std::min(C.n_closed(b), b_weight); };
  std::vector<int> w(L);
  std::vector<char> live(L, 1);
  for (int i = 0; i < L; ++i) w[i] = hw(idx[i]);
  std::vector<std::vector<int>> holders(C.nidx);
  for (int i = 0; i < L; ++i)
    idx[i].each([&](int x) { if (!C.keep.test(x)) holders[x].push_back(i); });
  std::extreme_value_distribution<double> gumbel(0.0, 1.0);
  int n_live = L;
  while (n_live > 1) {
    int ba = -1, bb = -1;
    double best = std::numeric_limits<double>::infinity();
    for (int x = 0; x < C.nidx; ++x) {
      auto& h = holders[x];
      if (h.size() != 2) continue;
      int a = h[0], b = h[1];
      if (!live[a] || !live[b] || a == b) continue;
      Bits m = C.merged(idx[a], idx[b]);
      double sc = std::ldexp(1.0, hw(m)), sa = std::ldexp(1.0, w[a]), sb = std::ldexp(1.0, w[b]);
      double cost = sc - alpha * (sa + sb);
      double key = std::copysign(std::log2(1.0 + std::fabs(cost)), cost);
      if (temperature > 0) key -= temperature * gumbel(rng);
      if (key < best) { best = key; ba = a; bb = b; }
    }
    if (ba < 0) {
      std::vector<int> lv;
      for (int i = 0; i < int(idx.size()); ++i) if (live[i]) lv.push_back(i);
      std::sort(lv.begin(), lv.end(), [&](int a, int b) { return w[a] < w[b]; });
      ba = lv[0];
      bb = lv[1];
    }
    Bits m = C.merged(idx[ba], idx[bb]);
    int id = int(idx.size());
    idx.push_back(m);
    w.push_back(hw(m));
    live.push_back(1);
    live[ba] = live[bb] = 0;
    tree.left.push_back(ba);
    tree.right.push_back(bb);
    m.each([&](int x) {
      if (C.keep.test(x)) return;
      for (auto& hh : holders[x]) if (hh == ba || hh == bb) hh = id;
    });
    --n_live;
  }
  int N = int(idx.size());
  tree.parent.assign(N, -1);
  for (int i = 0; i < int(tree.left.size()); ++i) {
    tree.parent[tree.left[i]] = L + i;
    tree.parent[tree.right[i]] = L + i;
  }
}

// ------------------------------------------------- recursive bisection
// Builds a tree top-down: the leaves of a subtree are split in two by a
// balanced min-cut bisection (Fiduccia-Mattheyses passes from a random,
// time-ordered or qubit-ordered start), so each contraction joins two
// regions of the circuit that share few wires; small regions are finished
// greedily.
struct Partitioner {
  const Ctx& C;
  const Network& net;
  std::vector<Bits> idx;
  std::vector<std::vector<std::pair<int, int>>> adj;  // (neighbour, bits)
  std::vector<int> where;
  std::vector<char> out_leaf;   // holds a closed output leg
  std::mt19937_64& rng;
  double imbalance = 0.1;
  int mode = 0;
  int out_weight = 0;           // cut weight of the hyperedge over out_leaf
  int restarts = 3;
  Tree tree;

  Partitioner(const Ctx& c, const Network& n, const std::vector<Bits>& leaf_idx,
              const Bits& sliced, std::mt19937_64& r)
      : C(c), net(n), rng(r) {
    int L = int(leaf_idx.size());
    idx.resize(L);
    for (int i = 0; i < L; ++i) idx[i] = leaf_idx[i].andnot(sliced);
    adj.assign(L, {});
    where.assign(L, -1);
    out_leaf.assign(L, 0);
    for (int i = 0; i < L; ++i) out_leaf[i] = (idx[i] & C.closed).any();
    std::vector<std::vector<int>> holders(C.nidx);
    for (int i = 0; i < L; ++i)
      idx[i].each([&](int x) { if (!C.keep.test(x)) holders[x].push_back(i); });
    for (int x = 0; x < C.nidx; ++x)
      if (holders[x].size() == 2) {
        int u = holders[x][0], v = holders[x][1];
        adj[u].push_back({v, C.bits_of[x]});
        adj[v].push_back({u, C.bits_of[x]});
      }
    tree.n_leaves = L;
  }

  int new_node(int a, int b) {
    tree.left.push_back(a);
    tree.right.push_back(b);
    return tree.n_leaves + int(tree.left.size()) - 1;
  }

  int small(const std::vector<int>& S) {
    std::vector<int> ids(S);
    std::vector<Bits> sets;
    for (int v : S) sets.push_back(idx[v]);
    while (ids.size() > 1) {
      int ba = 0, bb = 1;
      long best = LONG_MAX;
      for (size_t i = 0; i < ids.size(); ++i)
        for (size_t j = i + 1; j < ids.size(); ++j) {
          Bits m = C.merged(sets[i], sets[j]);
          bool share = (sets[i] & sets[j]).andnot(C.keep).any();
          long key = (share ? 0 : (1L << 40)) + (long(C.weight(m)) << 16) -
                     std::max(C.weight(sets[i]), C.weight(sets[j]));
          if (key < best) { best = key; ba = int(i); bb = int(j); }
        }
      Bits m = C.merged(sets[ba], sets[bb]);
      int id = new_node(ids[ba], ids[bb]);
      ids.erase(ids.begin() + bb);
      sets.erase(sets.begin() + bb);
      ids[ba] = id;
      sets[ba] = m;
    }
    return ids[0];
  }

  // cut weight of a bisection
  int cut(const std::vector<int>& S, const std::vector<char>& side) {
    const int n = int(S.size());
    for (int i = 0; i < n; ++i) where[S[i]] = i;
    int c = 0, o0 = 0, o1 = 0;
    for (int i = 0; i < n; ++i) {
      for (auto [j, w] : adj[S[i]]) {
        int lj = where[j];
        if (lj > i && side[lj] != side[i]) c += w;
      }
      if (out_leaf[S[i]]) (side[i] ? o1 : o0)++;
    }
    for (int i = 0; i < n; ++i) where[S[i]] = -1;
    if (o0 && o1) c += out_weight;
    return c;
  }

  void bisect(const std::vector<int>& S, std::vector<char>& side) {
    std::vector<char> best;
    int bc = INT_MAX;
    for (int r = 0; r < restarts; ++r) {
      std::vector<char> sd;
      bisect_once(S, sd, r);
      int c = cut(S, sd);
      if (c < bc) { bc = c; best = sd; }
    }
    side = best;
  }

  void bisect_once(const std::vector<int>& S, std::vector<char>& side, int restart) {
    const int n = int(S.size());
    side.assign(n, 0);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    if (mode == 0 || restart > 0) {
      std::shuffle(order.begin(), order.end(), rng);
    } else {
      std::uniform_int_distribution<int> jit(0, 2);
      std::vector<long> key(n);
      for (int i = 0; i < n; ++i) {
        const Leaf& lf = net.leaves[S[i]];
        key[i] = mode == 1 ? long(lf.t) * 4 + jit(rng) : long(lf.qa + lf.qb) * 4 + jit(rng);
      }
      std::sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    }
    const int lo = std::max(1, int(std::floor(n * (0.5 - imbalance))));
    const int hi = n - lo;
    for (int r = 0; r < n; ++r) side[order[r]] = r < n / 2 ? 0 : 1;
    for (int i = 0; i < n; ++i) where[S[i]] = i;
    for (int pass = 0; pass < 12; ++pass) {
      int cnt0 = 0;
      for (int i = 0; i < n; ++i) cnt0 += side[i] == 0;
      std::vector<int> gain(n, 0);
      for (int i = 0; i < n; ++i)
        for (auto [j, w] : adj[S[i]]) {
          int lj = where[j];
          if (lj < 0) continue;
          gain[i] += side[lj] != side[i] ? w : -w;
        }
      std::vector<char> locked(n, 0);
      std::vector<int> moves;
      int cum = 0, best = 0, best_len = 0;
      int ob[2] = {0, 0};
      for (int i = 0; i < n; ++i) if (out_leaf[S[i]]) ob[int(side[i])]++;
      for (int step = 0; step < n; ++step) {
        int bv = -1, bg = INT_MIN;
        for (int i = 0; i < n; ++i) {
          if (locked[i]) continue;
          int nc0 = cnt0 + (side[i] == 0 ? -1 : 1);
          if (nc0 < lo || nc0 > hi) continue;
          int g = gain[i];
          if (out_weight && out_leaf[S[i]]) {
            int ca = ob[int(side[i])], cb = ob[1 - int(side[i])];
            g += out_weight * (int(ca > 0 && cb > 0) - int(ca - 1 > 0));
          }
          if (g > bg) { bg = g; bv = i; }
        }
        if (bv < 0) break;
        int from = side[bv];
        if (out_leaf[S[bv]]) { ob[from]--; ob[1 - from]++; }
        side[bv] = 1 - from;
        cnt0 += from == 0 ? -1 : 1;
        locked[bv] = 1;
        gain[bv] = -gain[bv];
        for (auto [j, w] : adj[S[bv]]) {
          int lj = where[j];
          if (lj < 0) continue;
          gain[lj] += side[lj] == side[bv] ? -2 * w : 2 * w;
        }
        cum += bg;
        moves.push_back(bv);
        if (cum > best) { best = cum; best_len = int(moves.size()); }
      }
      for (int m = int(moves.size()) - 1; m >= best_len; --m) side[moves[m]] = 1 - side[moves[m]];
      if (best <= 0) break;
    }
    for (int i = 0; i < n; ++i) where[S[i]] = -1;
  }

  int build(const std::vector<int>& S) {
    if (S.size() == 1) return S[0];
    if (S.size() <= 10) return small(S);
    std::vector<char> side;
    bisect(S, side);
    std::vector<int> A, B;
    for (size_t i = 0; i < S.size(); ++i) (side[i] ? B : A).push_back(S[i]);
    if (A.empty() || B.empty()) return small(S);
    int a = build(A);
    int b = build(B);
    return new_node(a, b);
  }

  void run(Tree& out) {
    std::vector<int> all(tree.n_leaves);
    std::iota(all.begin(), all.end(), 0);
    build(all);
    int N = tree.n_leaves + int(tree.left.size());
    tree.parent.assign(N, -1);
    for (int i = 0; i < int(tree.left.size()); ++i) {
      tree.parent[tree.left[i]] = tree.n_leaves + i;
      tree.parent[tree.right[i]] = tree.n_leaves + i;
    }
    out = tree;
  }
};

// ------------------------------------------------------- tree evaluation
struct Eval {
  std::vector<Bits> idx;      // per node (unsliced)
  std::vector<Bits> closure;  // per node: all indices touched by its leaves
  std::vector<int> topo;      // internal nodes, children first
};

void post_order(const Tree& t, std::vector<int>& topo) {
  topo.clear();
  int N = t.n_leaves + int(t.left.size());
  if (N == t.n_leaves) return;
  int root = N - 1;
  for (int i = t.n_leaves; i < N; ++i) if (t.parent[i] < 0) root = i;
  std::vector<std::pair<int, int>> st{{root, 0}};
  while (!st.empty()) {
    auto& [n, s] = st.back();
    if (n < t.n_leaves) { st.pop_back(); continue; }
    int k = n - t.n_leaves;
    if (s == 0) { s = 1; st.push_back({t.left[k], 0}); }
    else if (s == 1) { s = 2; st.push_back({t.right[k], 0}); }
    else { topo.push_back(n); st.pop_back(); }
  }
}

void evaluate_sets(const Ctx& C, const std::vector<Bits>& leaf_idx, const Tree& t, Eval& e) {
  int L = t.n_leaves, N = L + int(t.left.size());
  e.idx.assign(N, Bits(C.nidx));
  e.closure.assign(N, Bits(C.nidx));
  for (int i = 0; i < L; ++i) { e.idx[i] = leaf_idx[i]; e.closure[i] = leaf_idx[i]; }
  post_order(t, e.topo);
  for (int n : e.topo) {
    int k = n - L;
    e.idx[n] = C.merged(e.idx[t.left[k]], e.idx[t.right[k]]);
    e.closure[n] = e.closure[t.left[k]] | e.closure[t.right[k]];
  }
}

struct Score {
  double total = 0;      // predicted time over all slices
  int max_w = 0;         // largest tensor of a slice, log2 elements
  double macs_var = 0, macs_inv = 0;
};

int step_dtype(int want, int chalf_min, int wa, int wb, int wc) {
  return (want == 1 && std::max(wc, std::max(wa, wb)) >= chalf_min) ? 1 : 0;
}

Score score(const Ctx& C, const Tree& t, const Eval& e, const Bits& sliced, int n_sliced,
            const CostFn& cf, int dtype, int chalf_min) {
  Score s;
  int L = t.n_leaves;
  double ns = std::ldexp(1.0, n_sliced);
  for (int i = 0; i < L; ++i) {
    Bits b = e.idx[i].andnot(sliced);
    s.max_w = std::max(s.max_w, C.plain_bits(b) + C.n_closed(b));
  }
  for (int n : e.topo) {
    int k = n - L;
    Bits As = e.idx[t.left[k]].andnot(sliced), Bs = e.idx[t.right[k]].andnot(sliced);
    Bits Cs = e.idx[n].andnot(sliced);
    Shape sh = C.classify(As, Bs);
    int wc = C.weight(Cs);
    int dt = step_dtype(dtype, chalf_min, C.weight(As), C.weight(Bs), wc);
    double c = cf.step(sh.wz, sh.wm, sh.wn, sh.wk, dt);
    double macs = std::ldexp(1.0, sh.wz + sh.wm + sh.wn + sh.wk);
    if ((e.closure[n] & sliced).any()) { s.total += c * ns; s.macs_var += macs; }
    else { s.total += c; s.macs_inv += macs; }
    s.max_w = std::max(s.max_w, wc);
  }
  return s;
}

// -------------------------------------------------------------- slicing
void greedy_slice(const Ctx& C, const Tree& t, const Eval& e, int cap, const CostFn& cf,
                  int dtype, int chalf_min, Bits& sliced, std::vector<int>& order,
                  int max_slices) {
  for (int it = 0; it < max_slices; ++it) {
    Score cur = score(C, t, e, sliced, int(order.size()), cf, dtype, chalf_min);
    if (cur.max_w <= cap) return;
    Bits cand(C.nidx);
    for (size_t n = 0; n < e.idx.size(); ++n)
      if (C.weight(e.idx[n].andnot(sliced)) > cap) cand = cand | e.idx[n];
    cand = cand.andnot(C.keep).andnot(sliced);
    // choose the wire that most reduces the summed excess over the cap of
    // all nodes, then the lowest total cost
    int bestx = -1;
    double bestv = std::numeric_limits<double>::infinity();
    cand.each([&](int x) {
      Bits s2 = sliced;
      s2.set(x);
      double excess = 0;
      for (size_t n = 0; n < e.idx.size(); ++n)
        excess += std::max(0, C.weight(e.idx[n].andnot(s2)) - cap);
      Score sc = score(C, t, e, s2, int(order.size()) + 1, cf, dtype, chalf_min);
      double v = excess * 1e3 + std::log2(sc.total);
      if (v < bestv) { bestv = v; bestx = x; }
    });
    if (bestx < 0) return;
    sliced.set(bestx);
    order.push_back(bestx);
  }
}

// --------------------------------------------------------- annealing
// Rotation at internal node P = (X, Y) with X = (X1, X2):
//   P = (X1, X') with X' = (X2, Y)   or   P = (X2, X') with X' = (X1, Y).
// Only X's leaf set and the steps of X and P change.
struct Annealer {
  const Ctx& C;
  Tree& t;
  Eval& e;
  const Bits& sliced;
  int ns;
  const CostFn& cf;
  int dtype, chalf_min, cap;

  double step_cost(const Bits& A, const Bits& B, const Bits& Cn, const Bits& clo) const {
    Bits As = A.andnot(sliced), Bs = B.andnot(sliced), Cs = Cn.andnot(sliced);
    Shape sh = C.classify(As, Bs);
    int dt = step_dtype(dtype, chalf_min, C.weight(As), C.weight(Bs), C.weight(Cs));
    double c = cf.step(sh.wz, sh.wm, sh.wn, sh.wk, dt);
    return (clo & sliced).any() ? c * std::ldexp(1.0, ns) : c;
  }
  double node_cost(int n) const {
    int k = n - t.n_leaves;
    return step_cost(e.idx[t.left[k]], e.idx[t.right[k]], e.idx[n], e.closure[n]);
  }

  void run(long iters, uint64_t seed, double T0, double T1) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const int L = t.n_leaves;
    const int NI = int(t.left.size());
    if (NI < 2) return;
    double total = 0;
    for (int n = L; n < L + NI; ++n) total += node_cost(n);
    for (long it = 0; it < iters; ++it) {
      double T = T0 * std::pow(T1 / T0, double(it) / double(std::max(1L, iters - 1)));
      int P = L + int(rng() % NI);
      int kp = P - L;
      int side = int(rng() % 2);
      int X = side == 0 ? t.left[kp] : t.right[kp];
      int Y = side == 0 ? t.right[kp] : t.left[kp];
      if (X < L) continue;
      int kx = X - L;
      int kind = int(rng() % 2);
      int X1 = t.left[kx], X2 = t.right[kx];
      int stay = kind == 0 ? X1 : X2;
      int moved = kind == 0 ? X2 : X1;
      Bits nX = C.merged(e.idx[moved], e.idx[Y]);
      if (C.weight(nX.andnot(sliced)) > cap) continue;
      Bits nXc = e.closure[moved] | e.closure[Y];
      double old_c = node_cost(X) + node_cost(P);
      double cx = step_cost(e.idx[moved], e.idx[Y], nX, nXc);
      double cp = step_cost(e.idx[stay], nX, e.idx[P], e.closure[P]);
      double new_total = total - old_c + cx + cp;
      double dlog = std::log(new_total) - std::log(total);
      if (dlog <= 0 || U(rng) < std::exp(-dlog / T)) {
        t.left[kx] = moved;
        t.right[kx] = Y;
        t.parent[moved] = X;
        t.parent[Y] = X;
        t.left[kp] = stay;
        t.right[kp] = X;
        t.parent[stay] = P;
        t.parent[X] = P;
        e.idx[X] = nX;
        e.closure[X] = nXc;
        total = new_total;
      }
    }
    post_order(t, e.topo);
  }
};

struct Candidate {
  Tree tree;
  Eval e;
  Bits sl;
  std::vector<int> order;
  double key = std::numeric_limits<double>::infinity();
};

}  // namespace

const CostFn& default_cost() {
  static FlopMem fm;
  return fm;
}

std::string plan_network(const Network& net, const PlanOptions& opt, HostPlan& hp,
                         const CostFn* rank_cost) {
  hp = HostPlan();
  // the search (candidate trees, annealing, slicing) runs on the FLOP +
  // memory cost; `rank_cost` (the learned model, when given) picks which of
  // the refined candidates, each a tree with its slicing, is kept.  Used
  // inside annealing or for the choice of sliced wires, the learned cost
  // steered the search to plans with more slices and a longer total time.
  const CostFn& cf = default_cost();
  const CostFn& rank_cf = rank_cost ? *rank_cost : default_cost();
  Ctx C(net);
  const int L = int(net.leaves.size());
  if (L < 2) return "network needs at least two tensors";
  if (C.nidx > MAX_INDICES) return "network has more indices than the planner supports";
  std::vector<Bits> leaf_idx(L, Bits(C.nidx));
  for (int i = 0; i < L; ++i)
    for (int x : net.leaves[i].idx) leaf_idx[i].set(x);
  const int cap = opt.max_log2;
  std::mt19937_64 rng(opt.seed);

  Bits forced(C.nidx);
  std::vector<int> forced_order;
  for (int x : opt.forced_slices) {
    if (x < 0 || x >= C.nidx || net.indices[x].kind != IDX_WIRE) return "forced sliced wire invalid";
    if (forced.test(x)) return "forced sliced wire repeated";
    forced.set(x);
    forced_order.push_back(x);
  }
  const bool fixed_slices = !opt.forced_slices.empty() || opt.n_sliced == 0;

  // 1. candidate trees, ranked by their cost with the forced slices only;
  //    the `restarts` best distinct ones are refined
  const int R = std::max(1, opt.restarts);
  std::vector<Candidate> top;   // ascending key, at most R
  auto offer = [&](const Tree& t) {
    Candidate c;
    c.sl = forced;
    c.order = forced_order;
    c.tree = t;
    evaluate_sets(C, leaf_idx, c.tree, c.e);
    Score s = score(C, c.tree, c.e, c.sl, int(c.order.size()), cf, opt.search_dtype, opt.chalf_min_log2);
    // over the cap only counts when the slices are fixed by the caller
    c.key = s.total + (fixed_slices && s.max_w > cap ? 1e30 * (s.max_w - cap) : 0);
    if (!std::isfinite(c.key)) return;
    for (const Candidate& o : top)
      if (o.key == c.key) return;   // the same tree found twice
    if (int(top.size()) == R && c.key >= top.back().key) return;
    auto at = std::upper_bound(top.begin(), top.end(), c.key,
                               [](double k, const Candidate& o) { return k < o.key; });
    top.insert(at, std::move(c));
    if (int(top.size()) > R) top.pop_back();
  };
  const double alphas[3] = {1.0, 0.5, 0.0};
  const int bws[3] = {net.nb, std::max(0, net.nb / 2), 0};
  for (int tr = 0; tr < opt.greedy_trials; ++tr) {
    double temp = tr < 3 ? 0.0 : 0.3 + 1.5 * double(tr % 7) / 6.0;
    Tree t;
    greedy_tree(C, leaf_idx, forced, rng, temp, alphas[(tr / 3) % 3], bws[tr % 3], t);
    offer(t);
    if (forced.any()) {  // the same search blind to the forced slices
      greedy_tree(C, leaf_idx, Bits(C.nidx), rng, temp, alphas[(tr / 3) % 3], bws[tr % 3], t);
      offer(t);
    }
  }
  const double imbs[4] = {0.05, 0.15, 0.3, 0.45};
  const int ows[3] = {0, net.nb, 4 * net.nb};
  for (int tr = 0; tr < opt.partition_trials; ++tr) {
    Partitioner pt(C, net, leaf_idx, forced, rng);
    pt.imbalance = imbs[tr % 4];
    pt.mode = (tr / 4) % 3;
    pt.out_weight = ows[(tr / 12) % 3];
    Tree t;
    pt.run(t);
    offer(t);
    if (forced.any()) {
      Partitioner pb(C, net, leaf_idx, Bits(C.nidx), rng);
      pb.imbalance = pt.imbalance;
      pb.mode = pt.mode;
      pb.out_weight = pt.out_weight;
      pb.run(t);
      offer(t);
    }
  }
  if (top.empty()) return "no tree found";

  // each refinement (annealing and slicing of one candidate, seeded by its
  // rank) is independent: run them on host threads, then keep the best by
  // the ranking cost (ties to the lower rank, so the result does not depend
  // on thread timing)
  const int nc = int(top.size());
  std::vector<std::string> errs(nc);
  std::vector<double> ranks(nc, std::numeric_limits<double>::infinity());
  auto refine = [&](int r) {
  const uint64_t rseed = opt.seed + 1000003ULL * uint64_t(r);
  std::string err;
  try {
  err = [&]() -> std::string {
  Candidate& best = top[r];
  // 2. anneal the candidate tree (half of the budget), with the forced slices
  const long sa_half = std::max(0L, opt.sa_iters / 2);
  auto current = [&]() {
    return score(C, best.tree, best.e, best.sl, int(best.order.size()), cf, opt.search_dtype,
                 opt.chalf_min_log2);
  };
  if (sa_half > 0) {
    int lim = fixed_slices ? std::max(cap, current().max_w) : INT_MAX / 4;
    Annealer an{C, best.tree, best.e, best.sl, int(best.order.size()), cf, opt.search_dtype,
                opt.chalf_min_log2, lim};
    an.run(sa_half, rseed + 101, 0.05, 0.002);
    evaluate_sets(C, leaf_idx, best.tree, best.e);
  }
  // 3. slice down to the cap: a few wires at a time, each round followed by
  //    annealing of the tree on the sliced network (never growing the widest
  //    tensor), so the tree adapts to the wires removed
  if (!fixed_slices) {
    const int per_round = 2;
    int rounds = 0;
    for (Score sc = current(); sc.max_w > cap; sc = current(), ++rounds) {
      if (int(best.order.size()) >= 62) return "no tree fits the memory cap within 62 sliced wires";
      int target = std::max(cap, sc.max_w - per_round);
      greedy_slice(C, best.tree, best.e, target, cf, opt.search_dtype, opt.chalf_min_log2, best.sl,
                   best.order, std::min(per_round, 62 - int(best.order.size())));
      if (sa_half > 0) {
        int lim = std::max(cap, current().max_w);
        Annealer an{C, best.tree, best.e, best.sl, int(best.order.size()), cf, opt.search_dtype,
                    opt.chalf_min_log2, lim};
        an.run(std::max(1L, sa_half / 16), rseed + 7 * rounds, 0.03, 0.002);
        evaluate_sets(C, leaf_idx, best.tree, best.e);
      }
    }
    // drop slices that are no longer needed
    bool changed = true;
    while (changed) {
      changed = false;
      Score cur = current();
      for (size_t i = 0; i < best.order.size(); ++i) {
        Bits s2 = best.sl;
        s2.reset(best.order[i]);
        Score sc = score(C, best.tree, best.e, s2, int(best.order.size()) - 1, cf, opt.search_dtype,
                         opt.chalf_min_log2);
        if (sc.max_w <= cap && sc.total < cur.total) {
          best.sl = s2;
          best.order.erase(best.order.begin() + i);
          changed = true;
          break;
        }
      }
    }
  }
  // at least n_sliced wires if asked for
  if (opt.n_sliced > 0 && opt.forced_slices.empty()) {
    while (int(best.order.size()) < opt.n_sliced) {
      Bits cand(C.nidx);
      for (auto& b : best.e.idx) cand = cand | b;
      cand = cand.andnot(C.keep).andnot(best.sl);
      int bx = -1;
      double bv = std::numeric_limits<double>::infinity();
      cand.each([&](int x) {
        Bits s2 = best.sl;
        s2.set(x);
        Score sc = score(C, best.tree, best.e, s2, int(best.order.size()) + 1, cf, opt.search_dtype,
                         opt.chalf_min_log2);
        if (sc.total < bv) { bv = sc.total; bx = x; }
      });
      if (bx < 0) return "not enough wires to slice";
      best.sl.set(bx);
      best.order.push_back(bx);
    }
  }
  Score fin = score(C, best.tree, best.e, best.sl, int(best.order.size()), cf, opt.search_dtype,
                    opt.chalf_min_log2);
  if (fin.max_w > cap) return "no tree fits the memory cap with the slices allowed";
  return std::string();
  }();
  } catch (const std::exception& ex) {
    err = std::string("planner refinement failed: ") + ex.what();
  }
  errs[r] = err;
  if (err.empty())
    ranks[r] = score(C, top[r].tree, top[r].e, top[r].sl, int(top[r].order.size()), rank_cf,
                     opt.search_dtype, opt.chalf_min_log2).total;
  };
  const int nthreads = std::max(1, std::min(nc, int(std::thread::hardware_concurrency())));
  if (nthreads == 1) {
    for (int r = 0; r < nc; ++r) refine(r);
  } else {
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t)
      pool.emplace_back([&]() {
        for (int r = next++; r < nc; r = next++) refine(r);
      });
    for (auto& th : pool) th.join();
  }
  Candidate best;
  best.sl = Bits(C.nidx);
  double best_rank = std::numeric_limits<double>::infinity();
  std::string first_err;
  for (int r = 0; r < nc; ++r) {
    if (!errs[r].empty()) {
      if (first_err.empty()) first_err = errs[r];
      continue;
    }
    if (ranks[r] < best_rank) {
      best_rank = ranks[r];
      best = std::move(top[r]);
    }
  }
  if (!std::isfinite(best_rank)) return first_err.empty() ? "no tree found" : first_err;
  Score fin = score(C, best.tree, best.e, best.sl, int(best.order.size()), cf, opt.search_dtype,
                    opt.chalf_min_log2);

  hp.tree = best.tree;
  hp.node_idx = best.e.idx;
  hp.sliced = best.order;
  hp.max_log2 = fin.max_w;
  const Bits& SL = best.sl;
  const Tree& T = hp.tree;

  // ------------------------------------------------------------ layout
  const int N = L + int(T.left.size());
  hp.order.assign(N, {});
  int root = N - 1;
  for (int i = L; i < N; ++i) if (T.parent[i] < 0) root = i;
  auto stored_batched = [&](int node) {
    return node >= L && C.batched(C.n_closed(best.e.idx[node]));
  };
  if (!stored_batched(root) && net.nb > 0) return "internal: root is not batched";
  hp.order[root] = net.root_order;
  {
    Bits rs = best.e.idx[root].andnot(SL).andnot(C.closed);
    Bits ro(C.nidx);
    for (int x : net.root_order) if (x != net.batch_index) ro.set(x);
    if (!(rs == ro)) return "internal: root indices differ from the output";
  }
  const std::vector<int>& topo = best.e.topo;
  std::vector<StepLayout> rev;
  for (auto it = topo.rbegin(); it != topo.rend(); ++it) {
    const int n = *it;
    const int k = n - L;
    int a = T.left[k], b = T.right[k];
    Bits As = best.e.idx[a].andnot(SL), Bs = best.e.idx[b].andnot(SL);
    const Shape sh = C.classify(As, Bs);
    {
      // A is the operand with the larger free side
      int fa = C.plain_bits(As) - sh.wk + (sh.batched ? 0 : C.n_closed(As));
      int fb = C.plain_bits(Bs) - sh.wk + (sh.batched ? 0 : C.n_closed(Bs));
      if (fa < fb) { std::swap(a, b); std::swap(As, Bs); }
    }
    const Bits kset = (As & Bs).andnot(C.keep);
    const std::vector<int>& oc = hp.order[n];
    std::vector<int> ml, nl, kl;
    bool has_b = false;
    for (int x : oc) {
      if (x == net.batch_index) { has_b = true; continue; }
      if (As.test(x)) ml.push_back(x);
      else if (Bs.test(x)) nl.push_back(x);
      else return "internal: result index not found in operands";
    }
    if (net.nb > 0 && sh.batched != has_b) return "internal: batch mismatch";
    kset.each([&](int x) { kl.push_back(x); });
    StepLayout s;
    s.a = a;
    s.b = b;
    s.out = n;
    s.batched = sh.batched;
    auto operand_order = [&](int node, const Bits& S, const std::vector<int>& free, Gather& g) {
      std::vector<int> o;
      if (s.batched) {
        if (stored_batched(node)) {
          g.stored_batched = true;
          if (net.batch_index >= 0) o.push_back(net.batch_index);
        } else {
          (S & C.closed).each([&](int x) { o.push_back(x); });
        }
      }
      o.insert(o.end(), free.begin(), free.end());
      o.insert(o.end(), kl.begin(), kl.end());
      if (s.batched && !g.stored_batched) {
        int64_t acc = 1;
        std::vector<int64_t> st(o.size());
        for (int i = int(o.size()) - 1; i >= 0; --i) { st[i] = acc; acc <<= C.bits_of[o[i]]; }
        for (size_t i = 0; i < o.size(); ++i)
          if (C.closed.test(o[i])) { g.q.push_back(net.indices[o[i]].q); g.stride.push_back(st[i]); }
      }
      return o;
    };
    hp.order[a] = operand_order(a, As, ml, s.ga);
    hp.order[b] = operand_order(b, Bs, nl, s.gb);
    std::vector<int64_t> cstride(C.nidx, 0);
    int64_t acc = 1;
    for (int i = int(oc.size()) - 1; i >= 0; --i) { cstride[oc[i]] = acc; acc <<= C.bits_of[oc[i]]; }
    auto expand = [&](const std::vector<int>& grp, std::vector<int64_t>& out) {
      for (int i = int(grp.size()) - 1; i >= 0; --i)
        for (int bt = 0; bt < C.bits_of[grp[i]]; ++bt) out.push_back(cstride[grp[i]] << bt);
    };
    if (s.batched && net.batch_index >= 0) expand({net.batch_index}, s.cz);
    expand(ml, s.cm);
    expand(nl, s.cn);
    s.nz = int(s.cz.size());
    s.nm = int(s.cm.size());
    s.nn = int(s.cn.size());
    for (int x : kl) s.nk += C.bits_of[x];
    s.variant = (best.e.closure[n] & SL).any();
    int wa = C.weight(As), wb = C.weight(Bs), wc = C.weight(best.e.idx[n].andnot(SL));
    s.dtype = step_dtype(opt.dtype, opt.exec_chalf_min_log2 >= 0 ? opt.exec_chalf_min_log2 : opt.chalf_min_log2,
                         wa, wb, wc);
    s.macs = std::ldexp(1.0, s.nz + s.nm + s.nn + s.nk);
    rev.push_back(s);
  }
  // A complex-half step whose B side is a narrow tensor (a gate or a small
  // branch: nn + nk <= 6 bits) keeps B in complex64: it runs on the
  // streaming kernel, which reads B once per row from cache, so B costs no
  // HBM traffic and is never rounded to half.
  for (auto& s : rev) {
    s.b_dtype = s.dtype;
    if (s.dtype == 1 && s.nn + s.nk <= 6) s.b_dtype = 0;
  }
  hp.steps.assign(rev.rbegin(), rev.rend());
  hp.step_of_node.assign(N, -1);
  for (size_t i = 0; i < hp.steps.size(); ++i) hp.step_of_node[hp.steps[i].out] = int(i);
  for (auto& s : hp.steps) {
    int par = T.parent[s.out];
    if (par < 0) { s.out_dtype = s.dtype; continue; }
    const StepLayout& c = hp.steps[hp.step_of_node[par]];
    s.out_dtype = s.out == c.b ? c.b_dtype : c.dtype;
  }
  for (auto& s : hp.steps) {
    auto es = [&](int node) {
      const StepLayout& c = hp.steps[hp.step_of_node[T.parent[node]]];
      return (node == c.b ? c.b_dtype : c.dtype) ? 4.0 : 8.0;
    };
    s.bytes = es(s.a) * std::ldexp(1.0, s.nz + s.nm + s.nk) +
              es(s.b) * std::ldexp(1.0, s.nz + s.nn + s.nk) +
              (s.out_dtype ? 4.0 : 8.0) * std::ldexp(1.0, s.nz + s.nm + s.nn);
    if (s.variant) { hp.macs_variant += s.macs; hp.bytes_variant += s.bytes; }
    else { hp.macs_invariant += s.macs; hp.bytes_invariant += s.bytes; }
  }
  // leaves carrying sliced wires: those on top, most significant bit first
  for (int i = 0; i < L; ++i) {
    std::vector<int> top;
    for (int t = int(best.order.size()) - 1; t >= 0; --t)
      if (leaf_idx[i].test(best.order[t])) top.push_back(best.order[t]);
    if (!top.empty()) {
      top.insert(top.end(), hp.order[i].begin(), hp.order[i].end());
      hp.order[i] = top;
    }
  }
  double ns = std::ldexp(1.0, int(best.order.size()));
  hp.log2_total_cost = std::log2(hp.macs_variant * ns + hp.macs_invariant + 1e-300);
  return "";
}

}  // namespace lf
