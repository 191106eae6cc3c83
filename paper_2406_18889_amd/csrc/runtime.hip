// Plan runtime and the extern "C" boundary (include/leapfrog.h).
//
// Workspace layout (one caller-owned device buffer, 256-byte aligned
// pieces):
//   [leaves]        every leaf tensor in full, in its storage type and layout
//   [slice leaves]  per-slice copies of the leaves that carry sliced wires
//   [invariant]     results of slice-independent subtrees (kept across slices)
//   [variant]       slice-dependent intermediates, packed by lifetime
//   [control]       slice counter, saturation counter, per-step amax
//   [tables]        slice-copy descriptors
//
// Complex-half scaling: every complex-half tensor T carries an integer
// exponent e_T with value = stored * 2^e_T.  Leaves get e from their largest
// entry.  For a step producing a complex-half tensor, the stored result is
// acc * 2^s where acc is the float32 accumulation of stored operands, and
// e_C = e_A + e_B - s.  The shift s of each step is calibrated once per plan
// on the first contracted slice by a pass that only records the largest
// |re|,|im| of acc, targeting 2^(16 - h) (h bits of headroom below the half
// range, h = 4 by default); later slices reuse it and count every value
// clamped to the half range.  Results stored as complex64 fold 2^(e_A + e_B)
// into their scale and carry e = 0.  The final sum into float64 multiplies
// by 2^e_root.
//
// Saturation: the accumulate kernel of a slice adds nothing once the plan's
// saturation counter is nonzero and records the smallest such slice number,
// so the caller's accumulator always holds a prefix of the requested range
// that saw no clamped value.  With check_overflow set, lf_contract_slices
// then either recalibrates the shifts on the first saturated slice with more
// headroom and contracts the rest of the range again, or reports
// LF_OVERFLOW (overflow_policy).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/leapfrog.h"
#include "kernels.h"
#include "plan.h"

namespace lf {
// costmodel.hip: the loaded learned cost, tabulated for batch exponent nb
// (nullptr when no model is loaded or its evaluation failed)
const CostFn* mlp_cost_fn_for(int nb, std::string* err);
}

namespace {
thread_local std::string g_err;
lf_status fail(lf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(LF_HIP_ERROR, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

constexpr int64_t ALIGN = 256;
int64_t align_up(int64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
}  // namespace

namespace lf {
// error reporting for the entry points of the other sources
lf_status set_error(lf_status s, const std::string& msg) { return fail(s, msg); }
}  // namespace lf

struct lf_plan {
  lf_plan_opts opts{};
  lf::Network net;
  lf::HostPlan hp;
  int n_nodes = 0;
  int root = -1;
  // per node
  std::vector<int> store_dt;       // storage type
  std::vector<int64_t> elems;      // per-slice elements
  std::vector<int64_t> off;        // byte offset of the tensor a step reads
  std::vector<int64_t> full_off;   // leaves: byte offset of the full tensor
  std::vector<int> exp2;           // power-of-two exponent (complex-half)
  std::vector<int> shift;          // per step (complex-half results)
  std::vector<lf::SliceCopy> copies;
  std::vector<int64_t> gtab_off;   // per step: byte offset of [offA | offB] tables, -1 if none
  // batch entry z (contraction order) -> the caller's closed string; empty
  // when the two orders agree.  Its device copy (int64 per string) sits at
  // off_rows and maps root rows to out_amps rows.
  std::vector<int64_t> batch_src;
  int64_t off_rows = -1;
  // grouped launches of small independent streaming steps: (first position
  // in variant_steps, step count, blocks, first table entry); built after
  // tuning and calibration for one generation and one timed kernel, the
  // tables in the workspace at off_groups
  struct Group { int first, count; int64_t blocks; int tab; };
  std::vector<Group> groups;
  std::vector<int> group_at;          // per position in variant_steps: group starting there, or -1
  std::vector<lf::GroupStep> group_tab;
  uint64_t groups_gen = ~0ull;
  int groups_time_kernel = -2;
  int64_t off_groups = 0;
  int64_t copy_max_n = 0;
  int64_t off_copies_tab = 0, off_sigma = 0, off_sat = 0, off_amax = 0;
  // off_sat holds the saturation counter (uint32) and, 8 bytes on, the first
  // slice left out because of it (uint64, all ones = none)
  uint64_t ws_bytes = 0;
  std::vector<int> variant_steps, invariant_steps;
  // binding
  char* ws = nullptr;
  uint64_t ws_size = 0;
  bool bound = false;
  bool invariant_done = false;
  bool calibrated = false;
  bool tuned = false;
  int headroom = 4;                  // calibration target 2^(16 - headroom)
  int recalibrations = 0;            // automatic recalibrations since bind
  uint64_t generation = 0;           // bumped whenever recorded launches go stale
  float slice_ms = -1.0f;            // measured time of one slice's steps (batch lane balance)
  std::string tune_path;             // autotune_cache of the options (empty: none)
  // graph cache
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  void* graph_out = nullptr;
  hipStream_t graph_stream = nullptr;
  int graph_slices = 0;
  hipStream_t cap_stream = nullptr;  // private stream used only to record graphs
  // live timing of one kernel's launches in stream-mode contractions
  int time_kernel = -1;
  std::vector<hipEvent_t> tev;       // event pool, two per timed launch
  std::vector<int> tev_step;         // step of each pair in use
  size_t tev_used = 0;               // pairs in use
  ~lf_plan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
  }
};

namespace {

using namespace lf;

int leaf_count(const lf_plan* p) { return p->hp.tree.n_leaves; }

unsigned* sat_ptr(const lf_plan* P) { return reinterpret_cast<unsigned*>(P->ws + P->off_sat); }
unsigned long long* first_bad_ptr(const lf_plan* P) {
  return reinterpret_cast<unsigned long long*>(P->ws + P->off_sat + 8);
}

// drops the process-wide batch graph if it records launches of P
void release_batch_graph_of(lf_plan* P);

// recorded launches (the plan's slice graph, a batch graph) carry shifts,
// scales and addresses as kernel arguments: drop them when those change
void drop_plan_graph(lf_plan* P) {
  if (P->graph_exec) { (void)hipGraphExecDestroy(P->graph_exec); P->graph_exec = nullptr; }
  if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
  P->generation++;
  release_batch_graph_of(P);
}

// Saturation state of the plan: the counter and the first slice left out.
// Synchronizes the stream.
lf_status read_sat(lf_plan* P, hipStream_t st, unsigned* sat, uint64_t* first_bad) {
  unsigned char buf[16];
  HIPCHK(hipMemcpyAsync(buf, P->ws + P->off_sat, sizeof(buf), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(sat, buf, 4);
  std::memcpy(first_bad, buf + 8, 8);
  return LF_OK;
}

lf_status clear_sat(lf_plan* P, hipStream_t st) {
  HIPCHK(launch_zero_u32(sat_ptr(P), 1, st));
  HIPCHK(launch_set_i64(reinterpret_cast<int64_t*>(first_bad_ptr(P)), -1, st));
  return LF_OK;
}

// -------------------------------------------------------- memory planning
// Contraction order of the closed strings.  A gathered operand of a batched
// step has one block per value of its closed bits, so strings that agree on
// those bits read the same block; sorted so that such strings are
// neighbours, the reads of one block follow each other and hit in cache
// instead of going to HBM once per string.  Sort key: the closed qubits of
// the gathered operands, the operand with the most gathered elements per
// slice first (slice-invariant steps last), within an operand by descending
// stride, so that strings next to each other also read blocks next to each
// other.  Padding entries (copies of string 0) stay at the end.
void order_batch(lf_plan* P) {
  Network& net = P->net;
  const int64_t B = net.n_batch;
  if (net.nb == 0 || B < 2) return;
  struct Op {
    double w;
    std::vector<std::pair<int64_t, int>> q;   // (stride, qubit)
  };
  std::vector<Op> ops;
  for (const StepLayout& st : P->hp.steps) {
    if (!st.batched) continue;
    auto add = [&](const Gather& g, int block_bits) {
      if (g.stored_batched || g.q.empty()) return;
      Op op;
      op.w = std::ldexp(1.0, st.nz + block_bits) * (st.variant ? 1.0 : 1e-12);
      for (size_t i = 0; i < g.q.size(); ++i) op.q.push_back({g.stride[i], g.q[i]});
      std::stable_sort(op.q.begin(), op.q.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
      ops.push_back(std::move(op));
    };
    add(st.ga, st.nm + st.nk);
    add(st.gb, st.nn + st.nk);
  }
  std::stable_sort(ops.begin(), ops.end(), [](const Op& x, const Op& y) { return x.w > y.w; });
  std::vector<int> bits;
  std::vector<char> used(64, 0);
  for (const Op& op : ops)
    for (const auto& sq : op.q)
      if (sq.second >= 0 && sq.second < 64 && !used[size_t(sq.second)]) {
        used[size_t(sq.second)] = 1;
        bits.push_back(sq.second);
      }
  if (bits.empty()) return;
  std::vector<uint64_t> key(size_t(B), 0);
  for (int64_t b = 0; b < B; ++b) {
    uint64_t k = 0;
    for (int q : bits) k = (k << 1) | ((net.closed_padded[size_t(b)] >> q) & 1);
    key[size_t(b)] = k;
  }
  std::vector<int64_t> perm(static_cast<size_t>(B));
  for (int64_t b = 0; b < B; ++b) perm[size_t(b)] = b;
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) { return key[size_t(x)] < key[size_t(y)]; });
  bool identity = true;
  for (int64_t z = 0; z < B && identity; ++z) identity = perm[size_t(z)] == z;
  if (identity) return;
  std::vector<uint64_t> given(net.closed_padded.begin(), net.closed_padded.begin() + B);
  for (int64_t z = 0; z < B; ++z) net.closed_padded[size_t(z)] = given[size_t(perm[size_t(z)])];
  P->batch_src = std::move(perm);
}

std::string plan_memory(lf_plan* P) {
  const HostPlan& hp = P->hp;
  const Network& net = P->net;
  const int L = hp.tree.n_leaves;
  const int N = L + int(hp.tree.left.size());
  P->n_nodes = N;
  P->root = N - 1;
  for (int i = 0; i < N; ++i) if (hp.tree.parent[i] < 0) P->root = i;
  std::vector<int> bits_of(net.indices.size());
  for (size_t i = 0; i < net.indices.size(); ++i) bits_of[i] = net.indices[i].bits;
  std::vector<char> is_sliced(net.indices.size(), 0);
  for (int x : hp.sliced) is_sliced[x] = 1;

  P->store_dt.assign(N, 0);
  P->elems.assign(N, 1);
  P->off.assign(N, -1);
  P->full_off.assign(N, -1);
  P->exp2.assign(N, 0);
  P->shift.assign(hp.steps.size(), 0);
  for (int n = 0; n < N; ++n) {
    int w = 0;
    for (int x : hp.order[n]) if (!is_sliced[x]) w += bits_of[x];
    P->elems[n] = int64_t(1) << w;
    int par = hp.tree.parent[n];
    if (par >= 0) {
      const StepLayout& c = hp.steps[hp.step_of_node[par]];
      P->store_dt[n] = n == c.b ? c.b_dtype : c.dtype;
    } else {
      P->store_dt[n] = n >= L ? hp.steps[hp.step_of_node[n]].out_dtype : 0;
    }
  }
  auto bytes_of = [&](int n) { return P->elems[n] * (P->store_dt[n] ? 4 : 8); };

  int64_t cur = 0;
  // leaves in full
  std::vector<int> n_sl(L, 0);
  for (int i = 0; i < L; ++i) {
    for (int x : hp.order[i]) if (is_sliced[x]) n_sl[i]++;
    int64_t b = bytes_of(i) << n_sl[i];
    P->full_off[i] = cur;
    cur += align_up(b);
  }
  // per-slice copies
  P->copies.clear();
  P->copy_max_n = 0;
  for (int i = 0; i < L; ++i) {
    if (!n_sl[i]) { P->off[i] = P->full_off[i]; continue; }
    P->off[i] = cur;
    SliceCopy c{};
    c.src = P->full_off[i];
    c.dst = cur;
    c.n = P->elems[i];
    c.es = P->store_dt[i] ? 4 : 8;
    c.nbits = n_sl[i];
    if (c.nbits > 8) return "a leaf carries more than 8 sliced wires";
    // sliced wires are the leading indices of the leaf layout
    int64_t stride = int64_t(c.es) * P->elems[i];
    for (int q = n_sl[i] - 1; q >= 0; --q) {
      int x = hp.order[i][q];
      int t = int(std::find(hp.sliced.begin(), hp.sliced.end(), x) - hp.sliced.begin());
      c.t[n_sl[i] - 1 - q] = t;
      c.stride[n_sl[i] - 1 - q] = stride;
      stride *= 2;
    }
    P->copies.push_back(c);
    P->copy_max_n = std::max(P->copy_max_n, c.n);
    cur += align_up(bytes_of(i));
  }
  // step classes
  P->variant_steps.clear();
  P->invariant_steps.clear();
  for (size_t s = 0; s < hp.steps.size(); ++s)
    (hp.steps[s].variant ? P->variant_steps : P->invariant_steps).push_back(int(s));
  // invariant results: permanent
  for (int s : P->invariant_steps) {
    int n = hp.steps[s].out;
    P->off[n] = cur;
    cur += align_up(bytes_of(n));
  }
  // variant results: interval packing over the per-slice step sequence
  struct Item { int node; int64_t bytes; int start, end; int64_t off; };
  std::vector<Item> items;
  std::vector<int> pos_of_step(hp.steps.size(), -1);
  for (size_t i = 0; i < P->variant_steps.size(); ++i) pos_of_step[P->variant_steps[i]] = int(i);
  const int nv = int(P->variant_steps.size());
  for (int s : P->variant_steps) {
    int n = hp.steps[s].out;
    int par = hp.tree.parent[n];
    int end = par < 0 ? nv : pos_of_step[hp.step_of_node[par]];
    items.push_back({n, align_up(bytes_of(n)), pos_of_step[s], end, -1});
  }
  std::vector<int> ordr(items.size());
  for (size_t i = 0; i < ordr.size(); ++i) ordr[i] = int(i);
  std::sort(ordr.begin(), ordr.end(), [&](int a, int b) { return items[a].bytes > items[b].bytes; });
  std::vector<int> placed;
  int64_t vpeak = 0;
  for (int i : ordr) {
    Item& it = items[i];
    std::vector<std::pair<int64_t, int64_t>> busy;
    for (int j : placed) {
      const Item& o = items[j];
      if (o.start <= it.end && it.start <= o.end) busy.push_back({o.off, o.off + o.bytes});
    }
    std::sort(busy.begin(), busy.end());
    int64_t at = 0;
    for (auto& b : busy) {
      if (at + it.bytes <= b.first) break;
      at = std::max(at, b.second);
    }
    it.off = at;
    placed.push_back(i);
    vpeak = std::max(vpeak, at + it.bytes);
  }
  for (auto& it : items) P->off[it.node] = cur + it.off;
  cur += align_up(vpeak);
  // gather tables of batched steps: 2^nb offsets for A, then for B
  P->gtab_off.assign(hp.steps.size(), -1);
  for (size_t s = 0; s < hp.steps.size(); ++s) {
    if (!hp.steps[s].batched) continue;
    P->gtab_off[s] = cur;
    cur += align_up(int64_t(2 * sizeof(int64_t)) << hp.steps[s].nz);
  }
  if (!P->batch_src.empty()) {
    P->off_rows = cur;
    cur += align_up(int64_t(sizeof(int64_t)) * int64_t(P->batch_src.size()));
  }
  // control block
  P->off_sigma = cur;
  cur += ALIGN;
  P->off_sat = cur;
  cur += ALIGN;
  P->off_amax = cur;
  cur += align_up(int64_t(sizeof(float)) * std::max<size_t>(1, hp.steps.size()));
  P->off_copies_tab = cur;
  cur += align_up(int64_t(sizeof(SliceCopy)) * std::max<size_t>(1, P->copies.size()));
  P->off_groups = cur;
  cur += align_up(int64_t(sizeof(GroupStep)) * std::max<size_t>(1, P->variant_steps.size()));
  P->ws_bytes = uint64_t(cur);
  return "";
}

// Leaf data in the stored layout (full, sliced wires leading), float64.
void leaf_layout(const lf_plan* P, int i, std::vector<cd>& out) {
  const Leaf& L = P->net.leaves[i];
  const std::vector<int>& ord = P->hp.order[i];
  const auto& ix = P->net.indices;
  // source strides (row-major over L.idx)
  std::vector<int64_t> sst(L.idx.size());
  int64_t acc = 1;
  for (int a = int(L.idx.size()) - 1; a >= 0; --a) { sst[a] = acc; acc <<= ix[L.idx[a]].bits; }
  int64_t n = acc;
  out.assign(n, cd(0));
  std::vector<int64_t> src_stride_of_dst(ord.size());
  std::vector<int> dbits(ord.size());
  for (size_t d = 0; d < ord.size(); ++d) {
    int a = int(std::find(L.idx.begin(), L.idx.end(), ord[d]) - L.idx.begin());
    src_stride_of_dst[d] = sst[a];
    dbits[d] = ix[ord[d]].bits;
  }
  for (int64_t e = 0; e < n; ++e) {
    int64_t rem = e, src = 0;
    for (int d = int(ord.size()) - 1; d >= 0; --d) {
      int64_t dim = int64_t(1) << dbits[d];
      src += (rem % dim) * src_stride_of_dst[d];
      rem /= dim;
    }
    out[e] = L.data[src];
  }
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Shape rule used until the autotuner has measured a shape.
int default_kernel(int dtype, int nz, int nm, int nn, int nk) {
  if (kernel_applicable(K_NARROW, dtype, nz, nm, nn, nk)) return K_NARROW;
  if (dtype == 1 && nk >= 3 && kernel_applicable(K_MFMA_BIG, dtype, nz, nm, nn, nk)) return K_MFMA_BIG;
  if (nk >= 2 && kernel_applicable(K_MFMA, dtype, nz, nm, nn, nk)) return K_MFMA;
  return K_THIN;
}

// Autotuner results shared by all plans of the process: fastest kernel per
// (nz, nm, nn, nk, compute type, result type).
std::mutex g_tune_mu;
std::map<std::array<int, 7>, int> g_tune;

GettArgs step_args(const lf_plan* P, int s) {
  const StepLayout& st = P->hp.steps[s];
  GettArgs a{};
  a.A = P->ws + P->off[st.a];
  a.B = P->ws + P->off[st.b];
  a.C = P->ws + P->off[st.out];
  a.nz = st.nz;
  a.nm = st.nm;
  a.nn = st.nn;
  a.nk = st.nk;
  if (P->gtab_off[s] >= 0) {
    a.offA = reinterpret_cast<const int64_t*>(P->ws + P->gtab_off[s]);
    a.offB = a.offA + (int64_t(1) << st.nz);
  }
  for (int i = 0; i < st.nz; ++i) a.cz[i] = st.cz[i];
  for (int i = 0; i < st.nm; ++i) a.cm[i] = st.cm[i];
  for (int i = 0; i < st.nn; ++i) a.cn[i] = st.cn[i];
  const int ea = P->exp2[st.a], eb = P->exp2[st.b];
  if (P->store_dt[st.out] == 1) a.scale = std::ldexp(1.0f, P->shift[s]);
  else a.scale = std::ldexp(1.0f, ea + eb);
  a.amax_only = 0;
  // the running maximum is recorded only by the calibration pass: one
  // atomic per wave on a single word serialises in L2 and would dominate
  // the time of streaming steps over millions of rows
  a.amax = nullptr;
  a.sat = reinterpret_cast<unsigned*>(P->ws + P->off_sat);
  return a;
}

lf_status run_step(lf_plan* P, int s, hipStream_t stream) {
  const StepLayout& st = P->hp.steps[s];
  GettArgs a = step_args(P, s);
  hipError_t e = launch_gett(st.kernel, P->store_dt[st.a], P->store_dt[st.b], P->store_dt[st.out], a, stream);
  if (e != hipSuccess) return fail(LF_HIP_ERROR, std::string("contraction launch: ") + hipGetErrorString(e));
  return LF_OK;
}

// propagate exponents in step order (complex64 results carry 0)
void propagate_exponents(lf_plan* P) {
  for (size_t s = 0; s < P->hp.steps.size(); ++s) {
    const StepLayout& st = P->hp.steps[s];
    if (P->store_dt[st.out] == 1) P->exp2[st.out] = P->exp2[st.a] + P->exp2[st.b] - P->shift[s];
    else P->exp2[st.out] = 0;
  }
}

// Calibrate the complex-half shifts on slice `sigma`: for each step in order
// whose result is stored in half, one pass records max |acc| without
// storing, then the shift is set and the step runs for real.
lf_status calibrate(lf_plan* P, int64_t sigma, hipStream_t stream) {
  drop_plan_graph(P);
  HIPCHK(launch_instantiate(reinterpret_cast<const SliceCopy*>(P->ws + P->off_copies_tab),
                            int(P->copies.size()), P->copy_max_n, P->ws, nullptr, sigma, stream));
  float* amax_dev = reinterpret_cast<float*>(P->ws + P->off_amax);
  for (size_t s = 0; s < P->hp.steps.size(); ++s) {
    const StepLayout& st = P->hp.steps[s];
    if (P->store_dt[st.out] == 1) {
      GettArgs a = step_args(P, int(s));
      a.scale = 1.0f;
      a.amax_only = 1;
      a.amax = amax_dev + s;
      HIPCHK(launch_zero_u32(reinterpret_cast<unsigned*>(amax_dev + s), 1, stream));
      HIPCHK(launch_gett(st.kernel, P->store_dt[st.a], P->store_dt[st.b], 1, a, stream));
      float mx = 0;
      HIPCHK(hipMemcpyAsync(&mx, amax_dev + s, sizeof(float), hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));
      int sh = 0;
      if (mx > 0 && std::isfinite(mx)) sh = (16 - P->headroom) - int(std::ceil(std::log2(double(mx))));
      P->shift[s] = sh;
      P->exp2[st.out] = P->exp2[st.a] + P->exp2[st.b] - sh;
    } else {
      P->exp2[st.out] = 0;
    }
    lf_status r = run_step(P, int(s), stream);
    if (r) return r;
  }
  P->calibrated = true;
  // a calibration pass leaves invariant results computed
  P->invariant_done = true;
  return LF_OK;
}

// grow the event pool so that `pairs` timed launches fit
lf_status reserve_events(lf_plan* P, size_t pairs) {
  while (P->tev.size() < 2 * pairs) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    P->tev.push_back(e);
  }
  if (P->tev_step.size() < pairs) P->tev_step.resize(pairs);
  return LF_OK;
}

// Groups of consecutive slice-dependent steps that run on the streaming
// kernel with at most 2^16 rows, none reading another's result or writing
// over another's operands (the per-slice allocation packs buffers by
// lifetime in step order, so a later step's result may take an earlier
// step's dead operand), at most 16 per group.  Each group becomes one launch
// of gett_thin_group; the steps' arguments are those of run_step.
lf_status build_groups(lf_plan* P, hipStream_t st) {
  P->groups.clear();
  P->group_tab.clear();
  const int nv = int(P->variant_steps.size());
  P->group_at.assign(size_t(nv), -1);
  auto esize = [&](int n) { return int64_t(P->store_dt[size_t(n)] == 1 ? 4 : 8); };
  auto overlap = [&](int x, int y) {
    const int64_t x0 = P->off[size_t(x)], x1 = x0 + P->elems[size_t(x)] * esize(x);
    const int64_t y0 = P->off[size_t(y)], y1 = y0 + P->elems[size_t(y)] * esize(y);
    return x0 < y1 && y0 < x1;
  };
  auto small = [&](int s) {
    const StepLayout& t = P->hp.steps[size_t(s)];
    return t.kernel == K_THIN && P->time_kernel != K_THIN && t.nz + t.nm <= 16;
  };
  if (P->opts.group_small_steps) {
    int i = 0;
    while (i < nv) {
      if (!small(P->variant_steps[size_t(i)])) { ++i; continue; }
      int j = i + 1;
      while (j < nv && j - i < 16 && small(P->variant_steps[size_t(j)])) {
        const StepLayout& b = P->hp.steps[size_t(P->variant_steps[size_t(j)])];
        bool ok = true;
        for (int k = i; k < j && ok; ++k) {
          const StepLayout& a = P->hp.steps[size_t(P->variant_steps[size_t(k)])];
          ok = b.a != a.out && b.b != a.out && !overlap(b.out, a.a) && !overlap(b.out, a.b) &&
               !overlap(b.out, a.out);
        }
        if (!ok) break;
        ++j;
      }
      if (j - i >= 2) {
        lf_plan::Group g{i, j - i, 0, int(P->group_tab.size())};
        for (int k = i; k < j; ++k) {
          const int s = P->variant_steps[size_t(k)];
          const StepLayout& t = P->hp.steps[size_t(s)];
          GroupStep e{};
          e.a = step_args(P, s);
          e.combo = P->store_dt[size_t(t.a)] | (P->store_dt[size_t(t.b)] << 1) | (P->store_dt[size_t(t.out)] << 2);
          e.blocks = thin_blocks(e.a);
          g.blocks += e.blocks;
          P->group_tab.push_back(e);
        }
        P->group_at[size_t(i)] = int(P->groups.size());
        P->groups.push_back(g);
      }
      i = j;
    }
  }
  if (!P->group_tab.empty()) {
    HIPCHK(hipMemcpyAsync(P->ws + P->off_groups, P->group_tab.data(), P->group_tab.size() * sizeof(GroupStep),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));   // the host table may change before the next build
  }
  P->groups_gen = P->generation;
  P->groups_time_kernel = P->time_kernel;
  return LF_OK;
}

bool groups_valid(const lf_plan* P) {
  return P->groups_gen == P->generation && P->groups_time_kernel == P->time_kernel;
}

// timed: bracket the launches of kernel P->time_kernel with events on the
// launch stream (stream mode only: events are not recorded into graphs)
lf_status run_slice(lf_plan* P, const int64_t* sigma_dev, int64_t sigma, double* out,
                    hipStream_t stream, bool timed = false) {
  HIPCHK(launch_instantiate(reinterpret_cast<const SliceCopy*>(P->ws + P->off_copies_tab),
                            int(P->copies.size()), P->copy_max_n, P->ws, sigma_dev, sigma, stream));
  const bool grouped = groups_valid(P);
  const int nv = int(P->variant_steps.size());
  for (int pos = 0; pos < nv; ++pos) {
    if (grouped && P->group_at[size_t(pos)] >= 0) {
      const lf_plan::Group& g = P->groups[size_t(P->group_at[size_t(pos)])];
      HIPCHK(launch_thin_group(reinterpret_cast<const GroupStep*>(P->ws + P->off_groups) + g.tab, g.count, g.blocks,
                               stream));
      pos += g.count - 1;
      continue;
    }
    const int s = P->variant_steps[size_t(pos)];
    const bool tk = timed && P->hp.steps[s].kernel == P->time_kernel;
    size_t pair = 0;
    if (tk) {
      pair = P->tev_used++;
      lf_status r = reserve_events(P, P->tev_used);
      if (r) return r;
      P->tev_step[pair] = s;
      HIPCHK(hipEventRecord(P->tev[2 * pair], stream));
    }
    lf_status r = run_step(P, s, stream);
    if (r) return r;
    if (tk) HIPCHK(hipEventRecord(P->tev[2 * pair + 1], stream));
  }
  const int r = P->root;
  const int lbits = int(P->net.open_qubits.size());
  const int64_t n = P->net.n_batch << lbits;
  const int64_t* rows = P->off_rows >= 0 ? reinterpret_cast<const int64_t*>(P->ws + P->off_rows) : nullptr;
  HIPCHK(launch_accumulate(P->store_dt[r], P->ws + P->off[r], out, n, lbits, rows,
                           std::ldexp(1.0, P->exp2[r]), sat_ptr(P), first_bad_ptr(P), sigma_dev,
                           sigma, stream));
  return LF_OK;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

void lf_plan_opts_default(lf_plan_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->dtype = LF_C64;
  o->max_log2_intermediate = 28;
  o->n_sliced_wires = -1;
  o->sliced_wires = nullptr;
  o->n_forced = 0;
  o->cost_model = LF_COST_FLOPMEM;
  o->greedy_trials = 8;
  o->partition_trials = 64;
  o->sa_iters = 0;
  o->seed = 1;
  o->chalf_min_log2 = 16;
  o->launch_mode = LF_LAUNCH_STREAM;
  o->check_overflow = 1;
  o->slices_per_graph = 8;
  o->search_dtype = -1;
  o->autotune = 1;
  o->restarts = 1;
  o->chalf_headroom_bits = 4;
  o->overflow_policy = LF_OVERFLOW_RECALIBRATE;
  o->chalf_exec_min_log2 = -1;
  o->mult = LF_MULT_AUTO;
  o->autotune_cache = nullptr;
  o->keep_batch_order = 0;
  o->group_small_steps = 1;
}

const char* lf_last_error(void) { return g_err.c_str(); }

lf_status lf_build_network(const lf_circuit* circuit, const int32_t* open_qubits, int32_t n_open,
                           const uint64_t* closed_bits, int64_t n_batch, const lf_plan_opts* opts,
                           lf_plan** out_plan) {
  try {
    if (!out_plan) return fail(LF_INVALID_ARGUMENT, "out_plan is NULL");
    *out_plan = nullptr;
    if (!circuit || (circuit->n_gates > 0 && !circuit->gates))
      return fail(LF_INVALID_ARGUMENT, "circuit is NULL");
    if (n_open < 0 || n_open > 30 || (n_open > 0 && !open_qubits))
      return fail(LF_INVALID_ARGUMENT, "n_open must be in [0, 30]");
    if (n_batch < 1 || !closed_bits) return fail(LF_INVALID_ARGUMENT, "need n_batch >= 1 closed strings");
    lf_plan_opts o;
    lf_plan_opts_default(&o);
    if (opts) o = *opts;
    if (o.dtype != LF_C64 && o.dtype != LF_CHALF) return fail(LF_INVALID_ARGUMENT, "dtype");
    if (o.search_dtype < -1 || o.search_dtype > LF_CHALF) return fail(LF_INVALID_ARGUMENT, "search_dtype");
    if (o.max_log2_intermediate < 1 || o.max_log2_intermediate > 34)
      return fail(LF_INVALID_ARGUMENT, "max_log2_intermediate must be in [1, 34]");
    if (o.launch_mode != LF_LAUNCH_STREAM && o.launch_mode != LF_LAUNCH_GRAPH)
      return fail(LF_INVALID_ARGUMENT, "launch_mode");
    if (o.slices_per_graph < 1 || o.slices_per_graph > 1024)
      return fail(LF_INVALID_ARGUMENT, "slices_per_graph must be in [1, 1024]");
    if (o.chalf_headroom_bits < -8 || o.chalf_headroom_bits > 24)
      return fail(LF_INVALID_ARGUMENT, "chalf_headroom_bits must be in [-8, 24]");
    if (o.overflow_policy != LF_OVERFLOW_RECALIBRATE && o.overflow_policy != LF_OVERFLOW_REPORT)
      return fail(LF_INVALID_ARGUMENT, "overflow_policy");
    std::vector<lf::GateIn> gates(circuit->n_gates);
    for (int g = 0; g < circuit->n_gates; ++g) {
      const lf_gate& G = circuit->gates[g];
      lf::GateIn& d = gates[g];
      d.nq = G.n_q;
      d.q[0] = G.q[0];
      d.q[1] = G.q[1];
      int dim = G.n_q == 1 ? 2 : 4;
      if (G.n_q != 1 && G.n_q != 2) return fail(LF_INVALID_ARGUMENT, "gate must act on 1 or 2 qubits");
      for (int e = 0; e < dim * dim; ++e) d.m[e] = lf::cd(G.mat[2 * e], G.mat[2 * e + 1]);
    }
    std::vector<int> openq(open_qubits, open_qubits + n_open);
    std::vector<uint64_t> cb(closed_bits, closed_bits + n_batch);
    if (o.mult == LF_MULT_3M)
      return fail(LF_INVALID_ARGUMENT, "mult: 3M complex products are not implemented (4M only)");
    if (o.mult != LF_MULT_AUTO && o.mult != LF_MULT_4M) return fail(LF_INVALID_ARGUMENT, "mult");
    auto P = std::make_unique<lf_plan>();
    P->opts = o;
    P->opts.autotune_cache = nullptr;   // the plan keeps its own copy of the path
    if (o.autotune_cache) {
      P->tune_path = o.autotune_cache;
      if (FILE* f = std::fopen(o.autotune_cache, "r")) {
        std::fclose(f);
        lf_status r = lf_autotune_load(o.autotune_cache);
        if (r) return r;
      }
    }
    std::string err = lf::build_network(circuit->n_qubits, gates, openq, cb, P->net);
    if (!err.empty()) return fail(LF_INVALID_ARGUMENT, err);
    lf::PlanOptions po;
    po.max_log2 = o.max_log2_intermediate;
    po.n_sliced = o.n_sliced_wires;
    po.greedy_trials = std::max(0, o.greedy_trials);
    po.partition_trials = std::max(0, o.partition_trials);
    if (po.greedy_trials + po.partition_trials < 1) po.greedy_trials = 1;
    po.sa_iters = long(std::max<int64_t>(0, o.sa_iters));
    po.seed = o.seed;
    po.cost_model = o.cost_model;
    po.dtype = o.dtype;
    po.search_dtype = o.search_dtype < 0 ? o.dtype : o.search_dtype;
    po.chalf_min_log2 = o.chalf_min_log2;
    if (o.chalf_exec_min_log2 < -1 || o.chalf_exec_min_log2 > 62)
      return fail(LF_INVALID_ARGUMENT, "chalf_exec_min_log2 must be -1 or in [0, 62]");
    po.exec_chalf_min_log2 = o.chalf_exec_min_log2;
    if (o.restarts < 1 || o.restarts > 64) return fail(LF_INVALID_ARGUMENT, "restarts must be in [1, 64]");
    po.restarts = o.restarts;
    if (o.n_forced > 0) {
      if (!o.sliced_wires) return fail(LF_INVALID_ARGUMENT, "sliced_wires is NULL");
      for (int t = 0; t < o.n_forced; ++t) {
        int id = P->net.wire_id(o.sliced_wires[2 * t], o.sliced_wires[2 * t + 1]);
        if (id < 0) return fail(LF_INVALID_ARGUMENT, "forced sliced wire is not an internal wire");
        po.forced_slices.push_back(id);
      }
    }
    const lf::CostFn* cf = nullptr;
    if (o.cost_model == LF_COST_MLP) {
      std::string e2;
      cf = lf::mlp_cost_fn_for(P->net.nb, &e2);
      if (!cf) {
        if (!e2.empty()) return fail(LF_HIP_ERROR, e2);
        return fail(LF_INVALID_ARGUMENT, "cost_model MLP requested but no model is loaded");
      }
    }
    err = lf::plan_network(P->net, po, P->hp, cf);
    if (!err.empty()) {
      if (err.find("cap") != std::string::npos) return fail(LF_PLAN_INFEASIBLE, err);
      return fail(LF_INTERNAL, err);
    }
    if (int(P->hp.sliced.size()) > 62) return fail(LF_PLAN_INFEASIBLE, "too many sliced wires");
    // default kernel choice
    for (auto& s : P->hp.steps) {
      s.kernel = default_kernel(s.dtype, s.nz, s.nm, s.nn, s.nk);
      if (s.b_dtype != s.dtype && s.kernel != lf::K_NARROW) s.kernel = lf::K_THIN;
    }
    for (auto& s : P->hp.steps)
      if (s.nz > lf::MAXZ || s.nm > lf::MAXMN || s.nn > lf::MAXMN)
        return fail(LF_PLAN_INFEASIBLE, "step rank exceeds kernel limits");
    if (!o.keep_batch_order) order_batch(P.get());
    err = plan_memory(P.get());
    if (!err.empty()) return fail(LF_PLAN_INFEASIBLE, err);
    *out_plan = P.release();
    return LF_OK;
  } catch (const std::exception& e) {
    return fail(LF_INTERNAL, e.what());
  }
}

lf_status lf_plan_get_info(const lf_plan* P, lf_plan_info* out) {
  if (!P || !out) return fail(LF_INVALID_ARGUMENT, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->n_sliced_wires = int32_t(P->hp.sliced.size());
  out->n_slices = int64_t(1) << P->hp.sliced.size();
  out->n_steps = int32_t(P->hp.steps.size());
  out->n_variant_steps = int32_t(P->variant_steps.size());
  out->n_leaves = P->hp.tree.n_leaves;
  out->max_log2_intermediate = P->hp.max_log2;
  out->dtype = P->opts.dtype;
  out->n_open = int32_t(P->net.open_qubits.size());
  out->n_batch = P->net.n_batch;
  out->n_batch_log2 = P->net.nb;
  int nh = 0;
  for (auto& s : P->hp.steps) nh += s.dtype;
  out->n_half_steps = nh;
  out->macs_per_slice = P->hp.macs_variant;
  out->macs_invariant = P->hp.macs_invariant;
  out->bytes_per_slice = P->hp.bytes_variant;
  out->bytes_invariant = P->hp.bytes_invariant;
  out->log2_total_macs = P->hp.log2_total_cost;
  out->workspace_bytes = P->ws_bytes;
  out->leaf_id_base = P->net.n2q + P->net.n_qubits;
  out->n_step_groups = int32_t(P->groups.size());
  out->n_grouped_steps = int32_t(P->group_tab.size());
  return LF_OK;
}

lf_status lf_plan_sliced_wires(const lf_plan* P, int32_t* qj) {
  if (!P || (!qj && !P->hp.sliced.empty())) return fail(LF_INVALID_ARGUMENT, "NULL argument");
  for (size_t t = 0; t < P->hp.sliced.size(); ++t) {
    const lf::Index& ix = P->net.indices[P->hp.sliced[t]];
    qj[2 * t] = ix.q;
    qj[2 * t + 1] = ix.j;
  }
  return LF_OK;
}

lf_status lf_plan_tree(const lf_plan* P, int32_t* leaf_canon, int32_t* left, int32_t* right) {
  if (!P || !leaf_canon || ((!left || !right) && !P->hp.steps.empty()))
    return fail(LF_INVALID_ARGUMENT, "NULL argument");
  const int L = P->hp.tree.n_leaves;
  const int base = P->net.n2q + P->net.n_qubits;
  for (int i = 0; i < L; ++i) leaf_canon[i] = P->net.leaves[i].canon_id;
  auto id = [&](int node) {
    return node < L ? P->net.leaves[node].canon_id : base + P->hp.step_of_node[node];
  };
  for (size_t s = 0; s < P->hp.steps.size(); ++s) {
    left[s] = id(P->hp.steps[s].a);
    right[s] = id(P->hp.steps[s].b);
  }
  return LF_OK;
}

lf_status lf_plan_steps(const lf_plan* P, int32_t* dims, double* macs, double* bytes) {
  if (!P || (!dims && !P->hp.steps.empty())) return fail(LF_INVALID_ARGUMENT, "NULL argument");
  for (size_t s = 0; s < P->hp.steps.size(); ++s) {
    const lf::StepLayout& st = P->hp.steps[s];
    int32_t* d = dims + 8 * s;
    d[0] = st.nz; d[1] = st.nm; d[2] = st.nn; d[3] = st.nk;
    d[4] = st.variant; d[5] = st.dtype; d[6] = P->store_dt[st.out]; d[7] = st.kernel;
    if (macs) macs[s] = st.macs;
    if (bytes) bytes[s] = st.bytes;
  }
  return LF_OK;
}

lf_status lf_plan_step_strides(const lf_plan* P, int32_t step, int64_t* out) {
  if (!P || !out || step < 0 || step >= int32_t(P->hp.steps.size())) return fail(LF_INVALID_ARGUMENT, "bad argument");
  const lf::StepLayout& st = P->hp.steps[step];
  int o = 0;
  for (auto v : st.cz) out[o++] = v;
  for (auto v : st.cm) out[o++] = v;
  for (auto v : st.cn) out[o++] = v;
  return LF_OK;
}

lf_status lf_plan_step_gather(const lf_plan* P, int32_t step, int32_t* info, int32_t* qa, int64_t* sa,
                              int32_t* qb, int64_t* sb) {
  if (!P || !info || step < 0 || step >= int32_t(P->hp.steps.size())) return fail(LF_INVALID_ARGUMENT, "bad argument");
  const lf::StepLayout& st = P->hp.steps[step];
  auto one = [&](const lf::Gather& g, int32_t* inf, int32_t* q, int64_t* s) {
    inf[0] = st.batched ? (g.stored_batched ? 1 : 0) : -1;
    inf[1] = st.batched ? int32_t(g.q.size()) : 0;
    inf[2] = 0;
    for (int i = 0; i < inf[1]; ++i) {
      if (q) q[i] = g.q[size_t(i)];
      if (s) s[i] = g.stride[size_t(i)];
    }
  };
  if (st.batched && (st.ga.q.size() > 64 || st.gb.q.size() > 64)) return fail(LF_INTERNAL, "gather wider than 64");
  one(st.ga, info, qa, sa);
  one(st.gb, info + 3, qb, sb);
  return LF_OK;
}

lf_status lf_plan_bind_workspace(lf_plan* P, void* dev_ptr, uint64_t bytes, void* stream) {
  if (!P) return fail(LF_INVALID_ARGUMENT, "plan is NULL");
  if (!dev_ptr) return fail(LF_INVALID_ARGUMENT, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % ALIGN) return fail(LF_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  if (bytes < P->ws_bytes) return fail(LF_OUT_OF_WORKSPACE, "workspace smaller than lf_plan_info.workspace_bytes");
  hipStream_t st = as_stream(stream);
  P->ws = static_cast<char*>(dev_ptr);
  P->ws_size = bytes;
  P->bound = false;
  P->invariant_done = false;
  P->calibrated = P->opts.dtype == LF_C64;
  P->headroom = P->opts.chalf_headroom_bits;
  P->recalibrations = 0;
  drop_plan_graph(P);
  // leaves: layout, exponent, rounding, upload
  const int L = leaf_count(P);
  std::vector<char> host;
  int64_t lo = P->full_off[0], hi = 0;
  for (int i = 0; i < L; ++i) {
    int64_t b = P->elems[i] * (P->store_dt[i] ? 4 : 8);
    int nsl = 0;
    for (int x : P->hp.order[i])
      if (std::find(P->hp.sliced.begin(), P->hp.sliced.end(), x) != P->hp.sliced.end()) nsl++;
    hi = std::max(hi, P->full_off[i] + (b << nsl));
  }
  host.assign(size_t(hi - lo), 0);
  std::vector<lf::cd> lay;
  for (int i = 0; i < L; ++i) {
    leaf_layout(P, i, lay);
    char* dst = host.data() + (P->full_off[i] - lo);
    if (P->store_dt[i] == 0) {
      float* f = reinterpret_cast<float*>(dst);
      for (size_t e = 0; e < lay.size(); ++e) { f[2 * e] = float(lay[e].real()); f[2 * e + 1] = float(lay[e].imag()); }
      P->exp2[i] = 0;
    } else {
      double mx = 0;
      for (auto& v : lay) mx = std::max(mx, std::max(std::fabs(v.real()), std::fabs(v.imag())));
      int e = mx > 0 ? int(std::ceil(std::log2(mx))) - 12 : 0;
      P->exp2[i] = e;
      _Float16* h = reinterpret_cast<_Float16*>(dst);
      for (size_t k = 0; k < lay.size(); ++k) {
        h[2 * k] = (_Float16)float(std::ldexp(lay[k].real(), -e));
        h[2 * k + 1] = (_Float16)float(std::ldexp(lay[k].imag(), -e));
      }
    }
  }
  if (P->opts.dtype == LF_C64) propagate_exponents(P);
  HIPCHK(hipMemcpyAsync(P->ws + lo, host.data(), host.size(), hipMemcpyHostToDevice, st));
  // gather tables
  std::vector<std::vector<int64_t>> tabs;
  for (size_t s = 0; s < P->hp.steps.size(); ++s) {
    if (P->gtab_off[s] < 0) continue;
    const lf::StepLayout& step = P->hp.steps[s];
    const int64_t Z = int64_t(1) << step.nz;
    std::vector<int64_t> t(2 * Z, 0);
    auto fill = [&](const lf::Gather& g, int64_t block, int64_t* out) {
      for (int64_t z = 0; z < Z; ++z) {
        if (g.stored_batched) { out[z] = z * block; continue; }
        const uint64_t cs = P->net.closed_padded[size_t(z)];
        int64_t o = 0;
        for (size_t i = 0; i < g.q.size(); ++i)
          if ((cs >> g.q[i]) & 1) o += g.stride[i];
        out[z] = o;
      }
    };
    fill(step.ga, int64_t(1) << (step.nm + step.nk), t.data());
    fill(step.gb, int64_t(1) << (step.nn + step.nk), t.data() + Z);
    tabs.push_back(std::move(t));
    HIPCHK(hipMemcpyAsync(P->ws + P->gtab_off[s], tabs.back().data(), 2 * Z * sizeof(int64_t),
                          hipMemcpyHostToDevice, st));
  }
  if (P->off_rows >= 0)
    HIPCHK(hipMemcpyAsync(P->ws + P->off_rows, P->batch_src.data(), P->batch_src.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, st));
  if (!P->copies.empty())
    HIPCHK(hipMemcpyAsync(P->ws + P->off_copies_tab, P->copies.data(),
                          P->copies.size() * sizeof(lf::SliceCopy), hipMemcpyHostToDevice, st));
  HIPCHK(lf::launch_zero_u32(sat_ptr(P), 1, st));
  HIPCHK(lf::launch_set_i64(reinterpret_cast<int64_t*>(first_bad_ptr(P)), -1, st));
  HIPCHK(lf::launch_zero_u32(reinterpret_cast<unsigned*>(P->ws + P->off_amax),
                             int64_t(std::max<size_t>(1, P->hp.steps.size())), st));
  // host staging buffer must outlive the copy
  HIPCHK(hipStreamSynchronize(st));
  P->bound = true;
  return LF_OK;
}

// Times every applicable kernel on each step of slice `sigma` (in step
// order, so every step reads real operands), keeps the fastest and leaves
// all results computed.
static lf_status autotune(lf_plan* P, int64_t sigma, hipStream_t st) {
  HIPCHK(launch_instantiate(reinterpret_cast<const SliceCopy*>(P->ws + P->off_copies_tab),
                            int(P->copies.size()), P->copy_max_n, P->ws, nullptr, sigma, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  lf_status r = LF_OK;
  for (size_t s = 0; s < P->hp.steps.size() && r == LF_OK; ++s) {
    StepLayout& stp = P->hp.steps[s];
    std::array<int, 7> key{stp.nz, stp.nm, stp.nn, stp.nk, P->store_dt[stp.a], P->store_dt[stp.b],
                           P->store_dt[stp.out]};
    int known = -1;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) known = it->second;
    }
    const bool mixed = P->store_dt[stp.a] != P->store_dt[stp.b];  // streaming kernels only
    if (known < 0) {
      float best = 1e30f;
      int bestk = stp.kernel;
      bool any_tile = false;
      for (int k = 1; k < K_COUNT; ++k)
        any_tile |= k != K_NARROW && kernel_applicable(k, stp.dtype, stp.nz, stp.nm, stp.nn, stp.nk);
      for (int k = 0; k < K_COUNT && r == LF_OK; ++k) {
        if (!kernel_applicable(k, stp.dtype, stp.nz, stp.nm, stp.nn, stp.nk)) continue;
        if (mixed && k != K_THIN && k != K_NARROW && k != K_SKINNY) continue;
        // the streaming kernel is a candidate only for a narrow side
        if (k == K_THIN && any_tile && stp.nn + stp.nk > 10) continue;
        stp.kernel = k;
        r = run_step(P, int(s), st);  // warm-up
        if (r) break;
        const int reps = stp.macs > 1e10 ? 2 : 5;
        if (hipEventRecord(e0, st) != hipSuccess) { r = fail(LF_HIP_ERROR, "event"); break; }
        for (int i = 0; i < reps && r == LF_OK; ++i) r = run_step(P, int(s), st);
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          r = fail(LF_HIP_ERROR, "event");
          break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; bestk = k; }
      }
      known = bestk;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = known;
    }
    stp.kernel = known;
    if (r == LF_OK) r = run_step(P, int(s), st);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r == LF_OK) P->tuned = true;
  if (r == LF_OK && !P->tune_path.empty()) r = lf_autotune_save(P->tune_path.c_str());
  return r;
}

static lf_status ensure_ready(lf_plan* P, int64_t sigma, hipStream_t st) {
  if (!P->calibrated) {
    lf_status r = calibrate(P, sigma, st);
    if (r) return r;
  }
  if (P->opts.autotune && !P->tuned) {
    lf_status r = autotune(P, sigma, st);
    if (r) return r;
    P->invariant_done = true;
  }
  if (!P->invariant_done) {
    for (int s : P->invariant_steps) {
      lf_status r = run_step(P, s, st);
      if (r) return r;
    }
    P->invariant_done = true;
  }
  if (!groups_valid(P)) {
    lf_status r = build_groups(P, st);
    if (r) return r;
  }
  return LF_OK;
}

static lf_status contract_graph(lf_plan* P, int64_t s0, int64_t count, double* out, hipStream_t st) {
  const int G = P->opts.slices_per_graph;
  int64_t* sigma_dev = reinterpret_cast<int64_t*>(P->ws + P->off_sigma);
  if (!P->graph_exec || P->graph_out != out || P->graph_slices != G) {
    if (P->graph_exec) { (void)hipGraphExecDestroy(P->graph_exec); P->graph_exec = nullptr; }
    if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
    // the caller's stream may be the null stream, which cannot be captured:
    // record on a private stream (nothing runs during capture), launch on st
    if (!P->cap_stream) HIPCHK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = P->cap_stream;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    lf_status r = LF_OK;
    for (int g = 0; g < G && r == LF_OK; ++g) {
      r = run_slice(P, sigma_dev, 0, out, cs);
      if (r == LF_OK && lf::launch_add_i64(sigma_dev, 1, cs) != hipSuccess)
        r = fail(LF_HIP_ERROR, "graph capture: counter kernel");
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (r) { if (g) (void)hipGraphDestroy(g); return r; }
    if (e != hipSuccess) return fail(LF_HIP_ERROR, std::string("end capture: ") + hipGetErrorString(e));
    P->graph = g;
    HIPCHK(hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0));
    P->graph_out = out;
    P->graph_stream = st;
    P->graph_slices = G;
  }
  int64_t done = 0;
  HIPCHK(lf::launch_set_i64(sigma_dev, s0, st));
  while (count - done >= G) {
    HIPCHK(hipGraphLaunch(P->graph_exec, st));
    done += G;
  }
  for (; done < count; ++done) {
    lf_status r = run_slice(P, nullptr, s0 + done, out, st);
    if (r) return r;
  }
  return LF_OK;
}

lf_status lf_contract_slices(lf_plan* P, int64_t s0, int64_t s1, void* out_amps, void* stream) {
  if (!P) return fail(LF_INVALID_ARGUMENT, "plan is NULL");
  if (!P->bound) return fail(LF_NOT_BOUND, "no workspace bound");
  const int64_t ns = int64_t(1) << P->hp.sliced.size();
  if (s0 < 0 || s1 < s0 || s1 > ns) return fail(LF_INVALID_ARGUMENT, "slice range outside [0, n_slices]");
  if (s0 == s1) return LF_OK;
  if (!out_amps) return fail(LF_INVALID_ARGUMENT, "out_amps is NULL");
  if (reinterpret_cast<uintptr_t>(out_amps) % 16) return fail(LF_INVALID_ARGUMENT, "out_amps not 16-byte aligned");
  hipStream_t st = as_stream(stream);
  double* out = static_cast<double*>(out_amps);
  lf_status r = ensure_ready(P, s0, st);
  if (r) return r;
  int64_t from = s0;
  for (int attempt = 0;; ++attempt) {
    if (P->opts.launch_mode == LF_LAUNCH_GRAPH && (s1 - from) >= P->opts.slices_per_graph) {
      r = contract_graph(P, from, s1 - from, out, st);
      if (r) return r;
    } else {
      for (int64_t s = from; s < s1; ++s) {
        r = run_slice(P, nullptr, s, out, st, P->time_kernel >= 0);
        if (r) return r;
      }
    }
    if (!P->opts.check_overflow) return LF_OK;
    unsigned sat = 0;
    uint64_t fb = ~uint64_t(0);
    r = read_sat(P, st, &sat, &fb);
    if (r) return r;
    if (!sat) return LF_OK;
    // out_amps holds [from, fb): every slice from fb on was left out
    const bool in_range = fb >= uint64_t(from) && fb < uint64_t(s1);
    if (!in_range || P->opts.overflow_policy == LF_OVERFLOW_REPORT || attempt == 3)
      return fail(LF_OVERFLOW, "complex-half values saturated: out_amps holds the slices before " +
                                   std::to_string(int64_t(fb)) + " (lf_plan_overflow)");
    // re-derive the shifts on the first saturated slice, two bits wider,
    // and contract the rest of the range again
    P->headroom = std::min(24, P->headroom + 2);
    P->recalibrations++;
    r = clear_sat(P, st);
    if (!r) r = calibrate(P, int64_t(fb), st);
    if (!r) r = clear_sat(P, st);
    if (r) return r;
    from = int64_t(fb);
  }
}

lf_status lf_plan_overflow(lf_plan* P, void* stream, lf_overflow_info* out, int32_t clear) {
  if (!P || !out) return fail(LF_INVALID_ARGUMENT, "NULL argument");
  if (!P->bound) return fail(LF_NOT_BOUND, "no workspace bound");
  hipStream_t st = as_stream(stream);
  unsigned sat = 0;
  uint64_t fb = ~uint64_t(0);
  lf_status r = read_sat(P, st, &sat, &fb);
  if (r) return r;
  std::memset(out, 0, sizeof(*out));
  out->saturated = sat;
  out->first_bad_slice = fb == ~uint64_t(0) ? -1 : int64_t(fb);
  out->recalibrations = P->recalibrations;
  out->headroom_bits = P->headroom;
  if (clear) {
    r = clear_sat(P, st);
    if (r) return r;
    HIPCHK(hipStreamSynchronize(st));
  }
  return LF_OK;
}

lf_status lf_plan_recalibrate(lf_plan* P, int64_t sigma, int32_t headroom_bits, void* stream) {
  if (!P) return fail(LF_INVALID_ARGUMENT, "plan is NULL");
  if (!P->bound) return fail(LF_NOT_BOUND, "no workspace bound");
  const int64_t ns = int64_t(1) << P->hp.sliced.size();
  if (sigma < 0 || sigma >= ns) return fail(LF_INVALID_ARGUMENT, "slice outside [0, n_slices)");
  if (headroom_bits < -8 || headroom_bits > 24)
    return fail(LF_INVALID_ARGUMENT, "headroom_bits must be in [-8, 24]");
  hipStream_t st = as_stream(stream);
  lf_status r = ensure_ready(P, sigma, st);
  if (r) return r;
  if (P->opts.dtype != LF_CHALF) return LF_OK;
  P->headroom = headroom_bits;
  r = calibrate(P, sigma, st);
  if (!r) r = clear_sat(P, st);
  if (r) return r;
  HIPCHK(hipStreamSynchronize(st));
  return LF_OK;
}

lf_status lf_debug_scale_slice_leaf(lf_plan* P, int32_t wire_bit, int32_t value, int32_t log2_factor,
                                    void* stream) {
  if (!P) return fail(LF_INVALID_ARGUMENT, "plan is NULL");
  if (!P->bound) return fail(LF_NOT_BOUND, "no workspace bound");
  if (wire_bit < 0 || wire_bit >= int32_t(P->hp.sliced.size()) || (value != 0 && value != 1) ||
      log2_factor < -60 || log2_factor > 60)
    return fail(LF_INVALID_ARGUMENT, "wire_bit, value or log2_factor out of range");
  // the first leaf whose per-slice copy depends on sliced wire `wire_bit`
  int leaf = -1;
  int64_t stride_elems = 0;
  for (const SliceCopy& c : P->copies) {
    for (int i = 0; i < c.nbits && leaf < 0; ++i)
      if (c.t[i] == wire_bit) {
        for (int l = 0; l < leaf_count(P); ++l)
          if (P->full_off[l] == c.src) leaf = l;
        stride_elems = c.stride[i] / c.es;
      }
    if (leaf >= 0) break;
  }
  if (leaf < 0) return fail(LF_INTERNAL, "no leaf carries that sliced wire");
  std::vector<cd> lay;
  leaf_layout(P, leaf, lay);
  const double f = std::ldexp(1.0, log2_factor);
  for (size_t e = 0; e < lay.size(); ++e)
    if (int64_t((int64_t(e) / stride_elems) & 1) == value) lay[e] *= f;
  std::vector<char> host;
  if (P->store_dt[leaf] == 0) {
    host.resize(lay.size() * 8);
    float* h = reinterpret_cast<float*>(host.data());
    for (size_t e = 0; e < lay.size(); ++e) { h[2 * e] = float(lay[e].real()); h[2 * e + 1] = float(lay[e].imag()); }
  } else {
    host.resize(lay.size() * 4);
    _Float16* h = reinterpret_cast<_Float16*>(host.data());
    for (size_t e = 0; e < lay.size(); ++e) {
      const double re = std::ldexp(lay[e].real(), -P->exp2[leaf]);
      const double im = std::ldexp(lay[e].imag(), -P->exp2[leaf]);
      if (std::fabs(re) > 65504.0 || std::fabs(im) > 65504.0)
        return fail(LF_INVALID_ARGUMENT, "factor takes a complex-half leaf outside the half range");
      h[2 * e] = (_Float16)float(re);
      h[2 * e + 1] = (_Float16)float(im);
    }
  }
  hipStream_t st = as_stream(stream);
  HIPCHK(hipMemcpyAsync(P->ws + P->full_off[leaf], host.data(), host.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return LF_OK;
}

namespace {
// Batched execution: the items are grouped into one chain per plan (a plan's
// workspace serialises its own slices), the chains are dealt to `lanes`
// lanes by their work, and each lane's chains are recorded as one graph
// that runs on a stream of its own.  A call forks the lanes from the
// caller's stream, launches one graph per lane and joins them back.  (One
// graph holding all lanes as parallel branches executes its branches one
// after another on this platform: 1.04x over sequential launches on the
// 512-subtask mix, against 2.06x for the same chains on four streams.)
struct BatchGraph {
  // (plan, its generation when recorded, slice range, accumulator) per item
  std::vector<std::tuple<lf_plan*, uint64_t, int64_t, int64_t, void*>> key;
  int lanes = 0;
  std::vector<hipGraph_t> graphs;      // per lane
  std::vector<hipGraphExec_t> execs;   // per lane
  std::vector<hipStream_t> streams;    // per lane, kept across recordings
  std::vector<hipEvent_t> events;      // fork event + one join event per lane
  void release() {
    for (auto& e : execs) (void)hipGraphExecDestroy(e);
    for (auto& g : graphs) (void)hipGraphDestroy(g);
    execs.clear();
    graphs.clear();
    lanes = 0;
  }
};
std::recursive_mutex g_batch_mu;
BatchGraph g_batch;

bool batch_uses(const BatchGraph& bg, const lf_plan* P) {
  for (auto& k : bg.key)
    if (std::get<0>(k) == P) return true;
  return false;
}

auto batch_key_of(const lf_batch_item& it) {
  return std::make_tuple(it.plan, it.plan->generation, it.slice_begin, it.slice_end, it.out_amps);
}

// time of one slice of P (slice copies and the slice-dependent steps, HIP
// events on `st`; the accumulator is not touched), measured once per plan
lf_status measure_slice(lf_plan* P, int64_t sigma, hipStream_t st) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  lf_status r = LF_OK;
  if (hipEventRecord(e0, st) != hipSuccess) r = fail(LF_HIP_ERROR, "event");
  if (r == LF_OK && launch_instantiate(reinterpret_cast<const SliceCopy*>(P->ws + P->off_copies_tab),
                                       int(P->copies.size()), P->copy_max_n, P->ws, nullptr, sigma, st) != hipSuccess)
    r = fail(LF_HIP_ERROR, "slice copy launch");
  for (size_t i = 0; r == LF_OK && i < P->variant_steps.size(); ++i) r = run_step(P, P->variant_steps[i], st);
  if (r == LF_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
    r = fail(LF_HIP_ERROR, "event");
  float ms = 0;
  if (r == LF_OK) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r == LF_OK) P->slice_ms = ms;
  return r;
}

// chains (items of one plan, in item order) dealt to lanes, heaviest chain
// first onto the least loaded lane (work: slices x the plan's measured time
// per slice)
std::vector<std::vector<int>> lane_items(const lf_batch_item* items, int n, int lanes) {
  std::vector<lf_plan*> order;
  std::map<lf_plan*, std::vector<int>> chains;
  std::map<lf_plan*, double> work;
  for (int i = 0; i < n; ++i) {
    lf_plan* P = items[i].plan;
    if (!chains.count(P)) order.push_back(P);
    chains[P].push_back(i);
    work[P] += double(items[i].slice_end - items[i].slice_begin) * std::max(1e-3, double(P->slice_ms));
  }
  std::stable_sort(order.begin(), order.end(), [&](lf_plan* a, lf_plan* b) { return work[a] > work[b]; });
  std::vector<std::vector<int>> out(lanes);
  std::vector<double> load(lanes, 0.0);
  for (lf_plan* P : order) {
    const int l = int(std::min_element(load.begin(), load.end()) - load.begin());
    load[l] += work[P];
    for (int i : chains[P]) out[l].push_back(i);
  }
  return out;
}

lf_status record_batch(const lf_batch_item* items, int n, int lanes, BatchGraph& bg) {
  bg.release();
  while (int(bg.streams.size()) < lanes) {
    hipStream_t s2;
    HIPCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    bg.streams.push_back(s2);
  }
  while (int(bg.events.size()) < lanes + 1) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    bg.events.push_back(e);
  }
  const std::vector<std::vector<int>> per_lane = lane_items(items, n, lanes);
  for (int l = 0; l < lanes; ++l) {
    hipStream_t ls = bg.streams[l];
    HIPCHK(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal));
    lf_status r = LF_OK;
    for (int i : per_lane[l])
      for (int64_t sg = items[i].slice_begin; sg < items[i].slice_end && r == LF_OK; ++sg)
        r = run_slice(items[i].plan, nullptr, sg, static_cast<double*>(items[i].out_amps), ls);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ls, &g);
    if (r || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      bg.release();
      if (r) return r;
      return fail(LF_HIP_ERROR, std::string("end capture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      bg.release();
      return fail(LF_HIP_ERROR, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    bg.graphs.push_back(g);
    bg.execs.push_back(ex);
  }
  bg.lanes = lanes;
  bg.key.clear();
  for (int i = 0; i < n; ++i) bg.key.push_back(batch_key_of(items[i]));
  return LF_OK;
}

// fork the lanes from `st`, one graph launch per lane, join back into `st`
lf_status launch_batch(BatchGraph& bg, hipStream_t st) {
  HIPCHK(hipEventRecord(bg.events[0], st));
  for (int l = 0; l < bg.lanes; ++l) {
    HIPCHK(hipStreamWaitEvent(bg.streams[l], bg.events[0], 0));
    HIPCHK(hipGraphLaunch(bg.execs[l], bg.streams[l]));
    HIPCHK(hipEventRecord(bg.events[1 + l], bg.streams[l]));
  }
  for (int l = 0; l < bg.lanes; ++l) HIPCHK(hipStreamWaitEvent(st, bg.events[1 + l], 0));
  return LF_OK;
}

void release_batch_graph_of(lf_plan* P) {
  std::lock_guard<std::recursive_mutex> lk(g_batch_mu);
  if (batch_uses(g_batch, P)) {
    g_batch.release();
    g_batch.key.clear();
  }
}

void forget_plan(lf_plan* P) {
  std::lock_guard<std::recursive_mutex> lk(g_batch_mu);
  release_batch_graph_of(P);
}

// After a batch: for every plan with check_overflow set, LF_OVERFLOW if its
// saturation counter is nonzero (synchronizes the stream).
lf_status batch_overflow(const lf_batch_item* items, int n, hipStream_t st) {
  std::vector<lf_plan*> seen;
  for (int i = 0; i < n; ++i) {
    lf_plan* P = items[i].plan;
    if (!P->opts.check_overflow || std::find(seen.begin(), seen.end(), P) != seen.end()) continue;
    seen.push_back(P);
    unsigned sat = 0;
    uint64_t fb = ~uint64_t(0);
    lf_status r = read_sat(P, st, &sat, &fb);
    if (r) return r;
    if (sat)
      return fail(LF_OVERFLOW, "complex-half values saturated in the batch (item " + std::to_string(i) +
                                   "): its plan's accumulator holds the slices before " +
                                   std::to_string(int64_t(fb)) + " in item order (lf_plan_overflow)");
  }
  return LF_OK;
}
}  // namespace

lf_status lf_contract_batch(const lf_batch_item* items, int32_t n, int32_t mode, int32_t lanes,
                            void* stream) {
  if (n < 0 || (n > 0 && !items)) return fail(LF_INVALID_ARGUMENT, "items");
  if (mode != LF_BATCH_SEQUENTIAL && mode != LF_BATCH_GRAPH) return fail(LF_INVALID_ARGUMENT, "mode");
  if (lanes < 0 || lanes > 8) return fail(LF_INVALID_ARGUMENT, "lanes must be in [0, 8]");
  hipStream_t st = as_stream(stream);
  for (int i = 0; i < n; ++i) {
    lf_plan* P = items[i].plan;
    if (!P) return fail(LF_INVALID_ARGUMENT, "item without a plan");
    if (!P->bound) return fail(LF_NOT_BOUND, "item plan has no workspace bound");
    const int64_t ns = int64_t(1) << P->hp.sliced.size();
    if (items[i].slice_begin < 0 || items[i].slice_end < items[i].slice_begin || items[i].slice_end > ns)
      return fail(LF_INVALID_ARGUMENT, "item slice range outside [0, n_slices]");
    if (!items[i].out_amps && items[i].slice_end > items[i].slice_begin)
      return fail(LF_INVALID_ARGUMENT, "item out_amps is NULL");
    if (reinterpret_cast<uintptr_t>(items[i].out_amps) % 16)
      return fail(LF_INVALID_ARGUMENT, "item out_amps not 16-byte aligned");
    lf_status r = ensure_ready(P, items[i].slice_begin, st);
    if (r) return r;
  }
  if (n == 0) return LF_OK;
  if (mode == LF_BATCH_SEQUENTIAL) {
    for (int i = 0; i < n; ++i)
      for (int64_t sg = items[i].slice_begin; sg < items[i].slice_end; ++sg) {
        lf_status r = run_slice(items[i].plan, nullptr, sg, static_cast<double*>(items[i].out_amps), st);
        if (r) return r;
      }
    return batch_overflow(items, n, st);
  }
  std::lock_guard<std::recursive_mutex> lk(g_batch_mu);
  std::vector<lf_plan*> pset;
  for (int i = 0; i < n; ++i) pset.push_back(items[i].plan);
  std::sort(pset.begin(), pset.end());
  pset.erase(std::unique(pset.begin(), pset.end()), pset.end());
  // lanes = 0: one lane per plan up to four (the hardware queues a process
  // gets by default); more lanes than plans would stay empty
  if (lanes == 0) lanes = std::min<int>(4, int(pset.size()));
  lanes = std::max(1, std::min<int>(lanes, int(pset.size())));
  bool same = !g_batch.execs.empty() && g_batch.lanes == lanes && int(g_batch.key.size()) == n;
  for (int i = 0; same && i < n; ++i) same = g_batch.key[i] == batch_key_of(items[i]);
  if (!same) {
    // lane balance needs each plan's time per slice (measured once)
    for (int i = 0; i < n; ++i)
      if (items[i].plan->slice_ms < 0) {
        lf_status r = measure_slice(items[i].plan, items[i].slice_begin, st);
        if (r) return r;
      }
    lf_status r = record_batch(items, n, lanes, g_batch);
    if (r) return r;
  }
  lf_status r = launch_batch(g_batch, st);
  if (r) return r;
  return batch_overflow(items, n, st);
}

lf_status lf_profile_steps(lf_plan* P, int32_t reps, double* out_ms, void* stream) {
  if (!P || !out_ms || reps < 1) return fail(LF_INVALID_ARGUMENT, "bad argument");
  if (!P->bound) return fail(LF_NOT_BOUND, "no workspace bound");
  hipStream_t st = as_stream(stream);
  lf_status r = ensure_ready(P, 0, st);
  if (r) return r;
  HIPCHK(lf::launch_instantiate(reinterpret_cast<const lf::SliceCopy*>(P->ws + P->off_copies_tab),
                                int(P->copies.size()), P->copy_max_n, P->ws, nullptr, 0, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (size_t s = 0; s < P->hp.steps.size(); ++s) {
    r = run_step(P, int(s), st);
    if (r) break;
    HIPCHK(hipEventRecord(e0, st));
    for (int i = 0; i < reps && r == LF_OK; ++i) r = run_step(P, int(s), st);
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    out_ms[s] = double(ms) / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return r;
}

lf_status lf_plan_time_kernel(lf_plan* P, int32_t kernel, int64_t reserve_launches) {
  if (!P) return fail(LF_INVALID_ARGUMENT, "plan is NULL");
  if (kernel < -1 || kernel >= lf::K_COUNT) return fail(LF_INVALID_ARGUMENT, "kernel id");
  if (reserve_launches < 0 || reserve_launches > (int64_t(1) << 20))
    return fail(LF_INVALID_ARGUMENT, "reserve_launches outside [0, 2^20]");
  P->time_kernel = kernel;
  P->tev_used = 0;
  return reserve_events(P, size_t(reserve_launches));
}

lf_status lf_plan_kernel_times(lf_plan* P, double* total_ms, int64_t* launches, double* per_step_ms,
                               int64_t* per_step_launches) {
  if (!P || !total_ms || !launches) return fail(LF_INVALID_ARGUMENT, "NULL pointer");
  const size_t ns = P->hp.steps.size();
  if (per_step_ms) std::fill(per_step_ms, per_step_ms + ns, 0.0);
  if (per_step_launches) std::fill(per_step_launches, per_step_launches + ns, int64_t(0));
  *total_ms = 0.0;
  *launches = int64_t(P->tev_used);
  if (P->tev_used) HIPCHK(hipEventSynchronize(P->tev[2 * P->tev_used - 1]));
  for (size_t i = 0; i < P->tev_used; ++i) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, P->tev[2 * i], P->tev[2 * i + 1]));
    *total_ms += ms;
    const int s = P->tev_step[i];
    if (per_step_ms) per_step_ms[s] += ms;
    if (per_step_launches) per_step_launches[s] += 1;
  }
  P->tev_used = 0;
  return LF_OK;
}

lf_status lf_autotune_save(const char* path) {
  if (!path) return fail(LF_INVALID_ARGUMENT, "path is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(LF_INVALID_ARGUMENT, std::string("cannot write ") + path);
  for (auto& kv : g_tune) {
    for (int x : kv.first) std::fprintf(f, "%d ", x);
    std::fprintf(f, "%d\n", kv.second);
  }
  std::fclose(f);
  return LF_OK;
}

lf_status lf_autotune_load(const char* path) {
  if (!path) return fail(LF_INVALID_ARGUMENT, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(LF_INVALID_ARGUMENT, std::string("cannot read ") + path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::array<int, 7> key;
  int k;
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d", &key[0], &key[1], &key[2], &key[3], &key[4],
                     &key[5], &key[6], &k) == 8) {
    if (k < 0 || k >= K_COUNT) continue;
    g_tune[key] = k;
  }
  std::fclose(f);
  return LF_OK;
}

lf_status lf_contract_pair(int32_t dtype_a, int32_t dtype_b, int32_t dtype_out, int32_t kernel,
                           const void* A, const void* B, void* C, int32_t nz, int32_t nm, int32_t nn,
                           int32_t nk, const int64_t* c_strides, float scale, void* stream) {
  if (!A || !B || !C || !c_strides) return fail(LF_INVALID_ARGUMENT, "NULL pointer");
  if ((dtype_a != 0 && dtype_a != 1) || (dtype_b != 0 && dtype_b != 1) || (dtype_out != 0 && dtype_out != 1))
    return fail(LF_INVALID_ARGUMENT, "dtype must be LF_C64 or LF_CHALF");
  if (dtype_a != dtype_b && !(dtype_a == 1 && dtype_b == 0))
    return fail(LF_INVALID_ARGUMENT, "mixed operands: only a complex-half A with a complex64 B");
  if (nz < 0 || nm < 0 || nn < 0 || nk < 0 || nz > lf::MAXZ || nm > lf::MAXMN || nn > lf::MAXMN ||
      nk > 40 || nz + nm + nk > 40 || nz + nn + nk > 40)
    return fail(LF_INVALID_ARGUMENT, "sizes out of range");
  if (reinterpret_cast<uintptr_t>(A) % 16 || reinterpret_cast<uintptr_t>(B) % 16)
    return fail(LF_INVALID_ARGUMENT, "A and B must be 16-byte aligned");
  if (kernel < -1 || kernel >= lf::K_COUNT) return fail(LF_INVALID_ARGUMENT, "kernel id");
  lf::GettArgs a{};
  a.A = A;
  a.B = B;
  a.C = C;
  a.nz = nz;
  a.nm = nm;
  a.nn = nn;
  a.nk = nk;
  for (int i = 0; i < nz; ++i) a.cz[i] = c_strides[i];
  for (int i = 0; i < nm; ++i) a.cm[i] = c_strides[nz + i];
  for (int i = 0; i < nn; ++i) a.cn[i] = c_strides[nz + nm + i];
  a.scale = scale;
  if (kernel < 0)
    kernel = lf::kernel_applicable(lf::K_MFMA, dtype_a, nz, nm, nn, nk) && nk >= 2 ? lf::K_MFMA : lf::K_THIN;
  HIPCHK(lf::launch_gett(kernel, dtype_a, dtype_b, dtype_out, a, as_stream(stream)));
  return LF_OK;
}

void lf_plan_destroy(lf_plan* P) {
  if (!P) return;
  forget_plan(P);
  delete P;
}

}  // extern "C"
