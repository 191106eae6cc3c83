// Host-side structures of the sliced tensor-network plan.
//
// The network (Methods A, C): gates become tensors; single-qubit gates are
// folded into two-qubit gate tensors in float64; |0> inputs are absorbed;
// output legs stay legs.  Open output legs belong to the result; a closed
// output leg is fixed, per sampled closed string b, to bit q of that string,
// which is done where a subtree first holds at least nb closed legs (nb =
// log2 of the batch padded to a power of two): from there on its tensor
// carries the batch index b instead of those legs (the partial "sparse
// state" of the final stem stages), and every later step is a batched
// product over b whose operands are gathered per b.  Every index is a bit
// (dimension 2) except b, which has dimension 2^nb.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace lf {

using cd = std::complex<double>;

enum IndexKind : int { IDX_WIRE = 0, IDX_OPEN = 1, IDX_CLOSED = 2, IDX_BATCH = 3 };

struct Index {
  int kind = IDX_WIRE;
  int q = -1;      // qubit (wire, open output)
  int j = -1;      // wire ordinal: point just before the j-th two-qubit gate on q
  int bits = 1;    // log2 of the dimension
};

// Small dense tensor used while building leaves, float64.
struct Leaf {
  int canon_id = -1;          // k-th two-qubit gate, or n2q + q for a gate-free qubit
  int qa = -1, qb = -1;       // qubits of the gate
  int t = 0;                  // position of the gate in the circuit
  std::vector<int> idx;       // index ids, idx[0] most significant
  std::vector<cd> data;       // row-major
};

// Fixed-width bitset over index ids (at most MAX_INDICES).
constexpr int MAX_INDICES = 1024;
struct Bits {
  static constexpr int W = MAX_INDICES / 64;
  uint64_t w[W];
  Bits() { for (int i = 0; i < W; ++i) w[i] = 0; }
  explicit Bits(int) : Bits() {}
  void set(int i) { w[i >> 6] |= 1ull << (i & 63); }
  void reset(int i) { w[i >> 6] &= ~(1ull << (i & 63)); }
  bool test(int i) const { return (w[i >> 6] >> (i & 63)) & 1; }
  bool any() const {
    uint64_t x = 0;
    for (int i = 0; i < W; ++i) x |= w[i];
    return x != 0;
  }
  int count() const {
    int c = 0;
    for (int i = 0; i < W; ++i) c += __builtin_popcountll(w[i]);
    return c;
  }
  Bits operator|(const Bits& o) const { Bits r; for (int i = 0; i < W; ++i) r.w[i] = w[i] | o.w[i]; return r; }
  Bits operator&(const Bits& o) const { Bits r; for (int i = 0; i < W; ++i) r.w[i] = w[i] & o.w[i]; return r; }
  Bits andnot(const Bits& o) const { Bits r; for (int i = 0; i < W; ++i) r.w[i] = w[i] & ~o.w[i]; return r; }
  bool operator==(const Bits& o) const {
    for (int i = 0; i < W; ++i) if (w[i] != o.w[i]) return false;
    return true;
  }
  template <class F> void each(F f) const {
    for (int i = 0; i < W; ++i) {
      uint64_t x = w[i];
      while (x) { int b = __builtin_ctzll(x); f(i * 64 + b); x &= x - 1; }
    }
  }
};

struct Network {
  int n_qubits = 0;
  int n2q = 0;
  int64_t n_batch = 1;         // closed strings requested
  int nb = 0;                  // log2 of the padded batch
  std::vector<int> open_qubits;
  std::vector<Index> indices;
  std::vector<Leaf> leaves;
  std::vector<int> wire_id_of;  // (q, j) -> index id lookup, flattened by wire_base
  std::vector<int> wire_base;   // per qubit
  std::vector<int> n2q_of;      // two-qubit gate count per qubit
  int batch_index = -1;         // id of b (used only by batched results), -1 if nb == 0
  std::vector<uint64_t> closed_padded;  // 2^nb closed strings (padding repeats string 0)
  std::vector<int> root_order;  // output layout: b, open[l-1] .. open[0]
  int wire_id(int q, int j) const;
};

struct GateIn {
  int nq;
  int q[2];
  cd m[16];
};

// Builds the canonical network.  Returns an error message or "".
std::string build_network(int n_qubits, const std::vector<GateIn>& gates,
                          const std::vector<int>& open_qubits,
                          const std::vector<uint64_t>& closed_bits, Network& net);

// ------------------------------------------------------------------ planning
enum CostModel : int { COST_FLOPMEM = 0, COST_MLP = 1 };

struct PlanOptions {
  int max_log2 = 28;           // cap on the elements of any sliced intermediate
  int n_sliced = -1;           // -1: planner decides from the cap
  std::vector<int> forced_slices;  // index ids to slice, in bit order
  int greedy_trials = 64;
  int partition_trials = 16;    // recursive min-cut bisection trees
  long sa_iters = 0;
  uint64_t seed = 1;
  int cost_model = COST_FLOPMEM;
  int dtype = 0;               // 0 complex64, 1 complex-half
  int search_dtype = 0;        // arithmetic whose step costs the search minimises
  int chalf_min_log2 = 16;     // tensors at least this large run in half
  int exec_chalf_min_log2 = -1;  // the same for the execution only; -1: chalf_min_log2
  int restarts = 1;            // best candidate trees refined; the ranking cost picks one
  double bytes_per_elem = 8.0;
};

struct Tree {
  int n_leaves = 0;                  // nodes [0, n_leaves) are leaves
  std::vector<int> left, right;      // per internal node (id - n_leaves)
  std::vector<int> parent;           // per node, -1 for the root
};

// Per-step description after layout.  Every index is expanded to bits.
// Operands are read as A[z][m][k] and B[z][n][k] (row-major, the last
// coordinate fastest); C is written through per-bit strides.
// In a batched step z runs over the 2^nb closed strings and each operand's
// [m][k] block for string z starts at an element offset from a table: a
// batched operand stores b on top (offset z 2^(m+k)); a plain operand still
// has closed legs on top and is gathered at the bits of string z.
struct Gather {
  bool stored_batched = false;
  std::vector<int> q;                // closed qubits (plain operand)
  std::vector<int64_t> stride;       // their element strides in the operand
};

struct StepLayout {
  int a = -1, b = -1, out = -1;      // node ids
  int nz = 0, nm = 0, nn = 0, nk = 0;
  bool batched = false;
  Gather ga, gb;
  std::vector<int64_t> cz, cm, cn;   // C element stride of each bit (bit 0 = lowest)
  bool variant = true;               // depends on the slice
  int dtype = 0;                     // compute type: 0 c64, 1 chalf
  int b_dtype = 0;                   // storage type of operand B (differs only for
                                     // a small B kept in complex64 beside a half A)
  int out_dtype = 0;
  double macs = 0, bytes = 0;
  int kernel = 0;                    // chosen variant (autotuner)
};

struct Plan;  // runtime plan, defined in runtime

// Plan search: tree + slicing + layout.
struct HostPlan {
  Tree tree;
  std::vector<Bits> node_idx;        // unsliced index sets
  std::vector<int> sliced;           // index ids, bit t of the slice number
  std::vector<std::vector<int>> order;  // per node: index ids, most significant first
  std::vector<StepLayout> steps;     // one per internal node, topological order
  std::vector<int> step_of_node;     // internal node -> position in steps
  int max_log2 = 0;                  // largest sliced intermediate (log2 elements)
  double macs_variant = 0, macs_invariant = 0;
  double bytes_variant = 0, bytes_invariant = 0;
  double log2_total_cost = 0;        // log2 of total MACs over all slices
};

struct CostFn;  // step cost callback

// rank_cost: cost that chooses among the refined candidates (null: the
// FLOP + memory cost that drives the search)
std::string plan_network(const Network& net, const PlanOptions& opt, HostPlan& hp,
                         const CostFn* rank_cost);

// Step cost used in the search: predicted time units of one step from its
// bit counts.  The default is FLOP + memory; the MLP model replaces it.
struct CostFn {
  virtual ~CostFn() {}
  virtual double step(int nz, int nm, int nn, int nk, int dtype) const = 0;
};

}  // namespace lf
