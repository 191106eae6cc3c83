// Canonical tensor network of a random circuit with a batch of closed
// output strings (Methods A: open qubits and correlated groups; Methods C:
// network simplified by the outcome bitstrings).
//
// Every two-qubit gate becomes one tensor.  The single-qubit gates between
// two two-qubit gates on a qubit are folded onto the output leg of the
// earlier one, so the leg between two gate tensors sits immediately before
// the later two-qubit gate; a qubit's leading single-qubit gates act on |0>
// and are folded onto the input leg of its first two-qubit gate.  Output
// legs stay as indices (open or closed); closed ones are fixed to the bits
// of each sampled string later, by the plan.  All arithmetic here is
// float64; the result is rounded once when leaves are uploaded.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "plan.h"

namespace lf {

namespace {

enum LegType { LEG_IDX = 0, LEG_OUT = 1 };
struct Leg {
  int type;
  int q;    // LEG_OUT: qubit
  int id;   // LEG_IDX: index id
  bool operator==(const Leg& o) const { return type == o.type && q == o.q && id == o.id; }
};

struct DT {
  std::vector<Leg> legs;
  std::vector<int> dims;
  std::vector<cd> d;
  int64_t size() const {
    int64_t s = 1;
    for (int x : dims) s *= x;
    return s;
  }
  std::vector<int64_t> strides() const {
    std::vector<int64_t> s(dims.size());
    int64_t acc = 1;
    for (int i = int(dims.size()) - 1; i >= 0; --i) { s[i] = acc; acc *= dims[i]; }
    return s;
  }
  int find(const Leg& l) const {
    for (size_t i = 0; i < legs.size(); ++i) if (legs[i] == l) return int(i);
    return -1;
  }
};

// t[..., x', ...] = sum_x m[x'][x] t[..., x, ...] on leg `pos` (dimension 2)
void apply_matrix(DT& t, int pos, const cd m[4]) {
  auto st = t.strides();
  int64_t s = st[pos], n = t.size();
  for (int64_t i = 0; i < n; ++i) {
    if ((i / s) % 2) continue;
    cd a0 = t.d[i], a1 = t.d[i + s];
    t.d[i] = m[0] * a0 + m[1] * a1;
    t.d[i + s] = m[2] * a0 + m[3] * a1;
  }
}

// removes leg `pos` by contracting it with the 2-vector v
void contract_vector(DT& t, int pos, const cd v[2]) {
  auto st = t.strides();
  DT r;
  for (size_t i = 0; i < t.legs.size(); ++i)
    if (int(i) != pos) { r.legs.push_back(t.legs[i]); r.dims.push_back(t.dims[i]); }
  r.d.assign(r.size(), cd(0));
  auto rs = r.strides();
  for (int64_t i = 0; i < r.size(); ++i) {
    int64_t rem = i, src = 0;
    int k = 0;
    for (size_t a = 0; a < t.legs.size(); ++a) {
      if (int(a) == pos) continue;
      int64_t c = rem / rs[k];
      rem %= rs[k];
      src += c * st[a];
      ++k;
    }
    r.d[i] = v[0] * t.d[src] + v[1] * t.d[src + st[pos]];
  }
  t = std::move(r);
}

}  // namespace

int Network::wire_id(int q, int j) const {
  if (q < 0 || q >= n_qubits) return -1;
  if (j < 1 || j >= n2q_of[q]) return -1;
  return wire_id_of[wire_base[q] + j];
}

std::string build_network(int n, const std::vector<GateIn>& gates,
                          const std::vector<int>& open_qubits,
                          const std::vector<uint64_t>& closed_bits, Network& net) {
  net = Network();
  if (n < 2 || n > 63) return "n_qubits must be in [2, 63]";
  net.n_qubits = n;
  std::vector<int> is_open(n, 0);
  for (int q : open_qubits) {
    if (q < 0 || q >= n) return "open qubit out of range";
    if (is_open[q]) return "duplicate open qubit";
    is_open[q] = 1;
  }
  net.open_qubits = open_qubits;
  int n_closed = n - int(open_qubits.size());
  if (closed_bits.empty()) return "need at least one closed string";
  net.n_batch = int64_t(closed_bits.size());
  if (n_closed == 0 && net.n_batch != 1) return "no closed qubits: batch must be 1";
  if (net.n_batch > (int64_t(1) << 22)) return "batch too large (max 2^22)";
  int nb = 0;
  while ((int64_t(1) << nb) < net.n_batch) ++nb;
  if (n_closed == 0) nb = 0;
  net.nb = nb;

  // pass 1: validate, count two-qubit gates per qubit
  net.n2q_of.assign(n, 0);
  for (size_t g = 0; g < gates.size(); ++g) {
    const GateIn& G = gates[g];
    if (G.nq == 1) {
      if (G.q[0] < 0 || G.q[0] >= n) return "gate qubit out of range";
    } else if (G.nq == 2) {
      if (G.q[0] < 0 || G.q[0] >= n || G.q[1] < 0 || G.q[1] >= n || G.q[0] == G.q[1])
        return "two-qubit gate qubits invalid";
      net.n2q_of[G.q[0]]++;
      net.n2q_of[G.q[1]]++;
      net.n2q++;
    } else {
      return "gate must act on 1 or 2 qubits";
    }
  }
  // index ids: internal wires (q, j), 1 <= j < J_q; open outputs; batch
  net.wire_base.assign(n, 0);
  int base = 0;
  for (int q = 0; q < n; ++q) { net.wire_base[q] = base; base += std::max(net.n2q_of[q], 1); }
  net.wire_id_of.assign(base, -1);
  for (int q = 0; q < n; ++q)
    for (int j = 1; j < net.n2q_of[q]; ++j) {
      Index ix; ix.kind = IDX_WIRE; ix.q = q; ix.j = j; ix.bits = 1;
      net.wire_id_of[net.wire_base[q] + j] = int(net.indices.size());
      net.indices.push_back(ix);
    }
  std::vector<int> out_id(n, -1);
  for (int q = 0; q < n; ++q) {
    Index ix; ix.kind = is_open[q] ? IDX_OPEN : IDX_CLOSED; ix.q = q; ix.bits = 1;
    out_id[q] = int(net.indices.size());
    net.indices.push_back(ix);
  }
  if (nb > 0) {
    Index ix; ix.kind = IDX_BATCH; ix.bits = nb;
    net.batch_index = int(net.indices.size());
    net.indices.push_back(ix);
  }
  net.closed_padded.assign(size_t(1) << nb, closed_bits[0]);
  for (size_t b = 0; b < closed_bits.size() && b < net.closed_padded.size(); ++b)
    net.closed_padded[b] = closed_bits[b];

  // pass 2: gate tensors
  const cd I2[4] = {1, 0, 0, 1};
  std::vector<std::array<cd, 4>> pending(n);
  for (int q = 0; q < n; ++q) std::copy(I2, I2 + 4, pending[q].begin());
  std::vector<int> count(n, 0), last(n, -1);
  std::vector<DT> ts;
  std::vector<std::array<int, 3>> coord;
  auto matmul2 = [](const cd* a, const std::array<cd, 4>& b) {
    std::array<cd, 4> r;
    r[0] = a[0] * b[0] + a[1] * b[2];
    r[1] = a[0] * b[1] + a[1] * b[3];
    r[2] = a[2] * b[0] + a[3] * b[2];
    r[3] = a[2] * b[1] + a[3] * b[3];
    return r;
  };
  auto out_leg = [&](int leaf, int q) {
    // the output leg of `leaf` on qubit q: a wire id or LEG_OUT
    int pos = ts[leaf].find(Leg{LEG_OUT, q, -1});
    if (pos >= 0) return pos;
    int j = count[q];  // this leaf was gate count[q]-1 on q; its out leg is wire (q, count[q])
    return ts[leaf].find(Leg{LEG_IDX, -1, net.wire_id(q, j)});
  };
  auto flush = [&](int q) {
    if (last[q] < 0) return;
    int pos = out_leg(last[q], q);
    apply_matrix(ts[last[q]], pos, pending[q].data());
    std::copy(I2, I2 + 4, pending[q].begin());
  };
  for (const GateIn& G : gates) {
    if (G.nq == 1) {
      int q = G.q[0];
      pending[q] = matmul2(G.m, pending[q]);
      continue;
    }
    int qa = G.q[0], qb = G.q[1];
    flush(qa);
    flush(qb);
    DT t;
    int qs[2] = {qa, qb};
    // legs: out_a, out_b, in_a, in_b ; matrix row = 2*out_a + out_b
    for (int s = 0; s < 2; ++s) {
      int q = qs[s];
      int j = count[q];
      Leg l;
      if (j == net.n2q_of[q] - 1) l = Leg{LEG_OUT, q, -1};
      else l = Leg{LEG_IDX, -1, net.wire_id(q, j + 1)};
      t.legs.push_back(l);
      t.dims.push_back(2);
    }
    for (int s = 0; s < 2; ++s) {
      int q = qs[s];
      int j = count[q];
      Leg l = (j == 0) ? Leg{LEG_OUT, -2 - q, -1} : Leg{LEG_IDX, -1, net.wire_id(q, j)};
      t.legs.push_back(l);
      t.dims.push_back(2);
    }
    t.d.assign(G.m, G.m + 16);
    // absorb |0> with leading single-qubit gates on first use of a qubit
    for (int s = 1; s >= 0; --s) {
      int q = qs[s];
      if (count[q] != 0) continue;
      int pos = t.find(Leg{LEG_OUT, -2 - q, -1});
      cd v[2] = {pending[q][0], pending[q][2]};  // pending * (1, 0)
      contract_vector(t, pos, v);
      std::copy(I2, I2 + 4, pending[q].begin());
    }
    int id = int(ts.size());
    ts.push_back(std::move(t));
    coord.push_back({qa, qb, int(&G - gates.data())});
    for (int s = 0; s < 2; ++s) { last[qs[s]] = id; count[qs[s]]++; }
  }
  // trailing single-qubit gates, gate-free qubits
  std::vector<int> canon(ts.size());
  for (size_t i = 0; i < ts.size(); ++i) canon[i] = int(i);
  for (int q = 0; q < n; ++q) {
    if (last[q] >= 0) {
      int pos = ts[last[q]].find(Leg{LEG_OUT, q, -1});
      apply_matrix(ts[last[q]], pos, pending[q].data());
    } else {
      DT t;
      t.legs.push_back(Leg{LEG_OUT, q, -1});
      t.dims.push_back(2);
      t.d = {pending[q][0], pending[q][2]};
      last[q] = int(ts.size());
      ts.push_back(std::move(t));
      canon.push_back(net.n2q + q);
      coord.push_back({q, q, int(gates.size())});
    }
  }
  // output legs: one index per qubit (open or closed)
  for (int q = 0; q < n; ++q) {
    DT& t = ts[last[q]];
    int pos = t.find(Leg{LEG_OUT, q, -1});
    if (pos < 0) return "internal: output leg missing";
    t.legs[pos] = Leg{LEG_IDX, -1, out_id[q]};
  }
  net.leaves.resize(ts.size());
  for (size_t i = 0; i < ts.size(); ++i) {
    Leaf& L = net.leaves[i];
    L.canon_id = canon[i];
    L.qa = coord[i][0];
    L.qb = coord[i][1];
    L.t = coord[i][2];
    for (auto& l : ts[i].legs) {
      if (l.type != LEG_IDX) return "internal: unresolved leg";
      L.idx.push_back(l.id);
    }
    L.data = std::move(ts[i].d);
  }
  // output layout: b, then open[l-1] ... open[0] (open[0] least significant)
  if (net.batch_index >= 0) net.root_order.push_back(net.batch_index);
  for (int i = int(open_qubits.size()) - 1; i >= 0; --i) net.root_order.push_back(out_id[open_qubits[i]]);
  return "";
}

}  // namespace lf
