// Host-side planning (see plan.hpp).  Fragments follow the paper's cutter
// output (Sec. V-A): disjoint subcircuits after cutting; roles of fragment
// inputs and outputs follow Sec. V-B.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <utility>

#include "../../include/ccut.h"

namespace ccut {

namespace {

bool is_two_qubit(uint32_t k) { return k == G_CX || k == G_CZ; }
bool is_clifford(uint32_t k) { return k <= G_CZ; }

struct DSU {
  std::vector<uint32_t> p;
  explicit DSU(size_t n) : p(n) { std::iota(p.begin(), p.end(), 0u); }
  uint32_t find(uint32_t a) {
    while (p[a] != a) {
      p[a] = p[p[a]];
      a = p[a];
    }
    return a;
  }
  void unite(uint32_t a, uint32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) p[a] = b;
  }
};

using cplx = std::complex<double>;
struct M2 {
  cplx a, b, c, d;  // [[a, b], [c, d]]
};
M2 mul(const M2 &L, const M2 &R) {  // L * R
  return {L.a * R.a + L.b * R.c, L.a * R.b + L.b * R.d, L.c * R.a + L.d * R.c, L.c * R.b + L.d * R.d};
}
M2 gate_matrix(uint32_t kind, double theta) {
  const double r = 1.0 / std::sqrt(2.0);
  const cplx i(0, 1);
  switch (kind) {
    case G_H: return {r, r, r, -r};
    case G_S: return {1, 0, 0, i};
    case G_SDG: return {1, 0, 0, -i};
    case G_X: return {0, 1, 1, 0};
    case G_Y: return {0, -i, i, 0};
    case G_Z: return {1, 0, 0, -1};
    case G_T: return {1, 0, 0, std::polar(1.0, M_PI / 4)};
    case G_TDG: return {1, 0, 0, std::polar(1.0, -M_PI / 4)};
    case G_RZ: return {1, 0, 0, std::polar(1.0, theta)};
    default: return {1, 0, 0, 1};
  }
}

// Fuse every run of one-qubit gates on a qubit (up to the next two-qubit
// gate touching it) into one matrix; runs on different qubits commute with
// the two-qubit gates that do not touch them, so emitting a run just before
// the first two-qubit gate on its qubit preserves the circuit.  A run that
// is diagonal so far also commutes with a CZ on its qubit and with a CX it
// controls, so it continues past them.
void fuse_one_qubit_runs(Fragment &F) {
  const uint32_t m = F.m();
  std::vector<M2> pend(m, M2{1, 0, 0, 1});
  std::vector<char> has(m, 0);
  auto flush = [&](uint32_t q) {
    if (!has[q]) return;
    const M2 &M = pend[q];
    F.sv_words.push_back(pack_op(G_U2, q, 0));
    const cplx e[4] = {M.a, M.b, M.c, M.d};
    for (auto &z : e) {
      F.sv_mats.push_back(z.real());
      F.sv_mats.push_back(z.imag());
    }
    pend[q] = M2{1, 0, 0, 1};
    has[q] = 0;
  };
  for (size_t g = 0; g < F.op_words.size(); ++g) {
    const uint32_t w = F.op_words[g], k = op_kind(w), a = op_q0(w), b = op_q1(w);
    if (is_two_qubit(k)) {
      // a diagonal run commutes with a CZ on its qubit and with a CX it
      // controls, so it stays pending and merges with the next run
      auto diag = [&](uint32_t q) { return pend[q].b == 0.0 && pend[q].c == 0.0; };
      if (!(diag(a) && (k == G_CZ || k == G_CX))) flush(a);
      if (!(diag(b) && k == G_CZ)) flush(b);
      F.sv_words.push_back(w);
      for (int t = 0; t < 8; ++t) F.sv_mats.push_back(0.0);
    } else {
      pend[a] = mul(gate_matrix(k, F.op_theta[g]), pend[a]);
      has[a] = 1;
    }
  }
  for (uint32_t q = 0; q < m; ++q) flush(q);
}

// Lay the fused stream out for the register-resident state-vector kernel
// (positions as in sv_shape).  Qubit q starts at position q.  Before an op
// that mixes amplitudes along a qubit that sits at a wave position, that
// qubit swaps places with the register or lane qubit whose next such use
// lies furthest ahead (Belady's rule), so swaps stay rare.  One-qubit
// unitaries with zero off-diagonal entries become SV_DIAG, which runs at any
// position.  The program ends with SV_END carrying the final layout.
void build_sv_program(Fragment &F) {
  const uint32_t m = F.m();
  const SvShape sh = sv_shape(m);
  const uint32_t inner = sh.rb + sh.lb;  // positions below this are register or lane bits
  const size_t n = F.sv_words.size();
  std::vector<int32_t> need(n, -1);
  std::vector<char> diag(n, 0);
  for (size_t g = 0; g < n; ++g) {
    const uint32_t w = F.sv_words[g], k = op_kind(w);
    if (k == G_U2) {
      const double *M = &F.sv_mats[8 * g];
      diag[g] = M[2] == 0.0 && M[3] == 0.0 && M[4] == 0.0 && M[5] == 0.0;
      if (!diag[g]) need[g] = (int32_t)op_q0(w);
    } else if (k == G_CX) {
      need[g] = (int32_t)op_q1(w);  // the target
    }
  }
  std::vector<std::vector<size_t>> uses(m);
  for (size_t g = 0; g < n; ++g)
    if (need[g] >= 0) uses[need[g]].push_back(g);
  std::vector<size_t> next(m, 0);
  auto next_use = [&](uint32_t q, size_t g) {  // first use after op g
    while (next[q] < uses[q].size() && uses[q][next[q]] <= g) ++next[q];
    return next[q] < uses[q].size() ? uses[q][next[q]] : SIZE_MAX;
  };
  std::vector<uint32_t> pos(m), at(m);
  for (uint32_t q = 0; q < m; ++q) pos[q] = at[q] = q;
  auto emit = [&](uint32_t kind, uint32_t a, uint32_t b, const double *M) {
    F.sv_prog.push_back(pack_op(kind, a, b));
    for (int t = 0; t < 8; ++t) F.sv_prog_mats.push_back(M ? M[t] : 0.0);
  };
  for (size_t g = 0; g < n; ++g) {
    const uint32_t w = F.sv_words[g], k = op_kind(w), a = op_q0(w), b = op_q1(w);
    if (k != G_U2 && k != G_CX && k != G_CZ) continue;
    if (need[g] >= 0 && pos[need[g]] >= inner) {
      const uint32_t q = (uint32_t)need[g];
      uint32_t victim = 0;
      size_t far = 0;
      for (uint32_t p = 0; p < inner; ++p) {
        const size_t u = next_use(at[p], g);
        if (p == 0 || u > far) {
          far = u;
          victim = p;
        }
      }
      const uint32_t pw = pos[q], qv = at[victim];
      emit(SV_SWAP, victim, pw, nullptr);
      std::swap(at[victim], at[pw]);
      pos[q] = victim;
      pos[qv] = pw;
    }
    if (k == G_U2)
      emit(diag[g] ? SV_DIAG : SV_U2, pos[a], 0, &F.sv_mats[8 * g]);
    else
      emit(k == G_CX ? SV_CX : SV_CZ, pos[a], pos[b], nullptr);
  }
  uint64_t layout = 0;
  for (uint32_t q = 0; q < m; ++q) layout |= (uint64_t)pos[q] << (4 * q);
  double M[8] = {};
  std::memcpy(&M[0], &layout, 8);
  emit(SV_END, 0, 0, M);
}

// Order a Clifford stream by ASAP layer: op g goes one layer after the
// latest earlier op on any of its qubits, so each layer acts on disjoint
// qubits and per-qubit order is kept (ops on disjoint qubits commute).
void layer_stream(std::vector<uint32_t> &words, std::vector<uint32_t> &starts, uint32_t m) {
  std::vector<int32_t> qlayer(m, -1);
  std::vector<uint32_t> lay(words.size());
  uint32_t nl = 0;
  for (size_t g = 0; g < words.size(); ++g) {
    const uint32_t w = words[g], k = op_kind(w), a = op_q0(w);
    const uint32_t b = (k == G_CX || k == G_CZ) ? op_q1(w) : a;
    const int32_t L = std::max(qlayer[a], qlayer[b]) + 1;
    lay[g] = (uint32_t)L;
    qlayer[a] = qlayer[b] = L;
    nl = std::max(nl, (uint32_t)L + 1);
  }
  starts.assign(nl + 1, 0);
  for (uint32_t L : lay) starts[L + 1]++;
  for (uint32_t L = 0; L < nl; ++L) starts[L + 1] += starts[L];
  std::vector<uint32_t> pos(starts.begin(), starts.end() - 1), out(words.size());
  for (size_t g = 0; g < words.size(); ++g) out[pos[lay[g]]++] = words[g];
  words.swap(out);
}

// Fuse every run of one-qubit Cliffords on a qubit into one G_C1 word,
// emitted just before the next two-qubit gate on that qubit (or at the
// end): the forward stream for tableau passes and, from the same runs, the
// reversed stream of inverse gates for the Heisenberg carry-back.
void fuse_clifford_runs(Fragment &F) {
  const uint32_t m = F.m();
  std::vector<uint32_t> fwd(m, 0u), inv(m, 0u);
  std::vector<char> has(m, 0);
  std::vector<uint32_t> back;  // built forward, reversed at the end
  auto flush = [&](uint32_t q) {
    if (!has[q]) return;
    F.cl_words.push_back(pack_op(G_C1, q, fwd[q]));
    back.push_back(pack_op(G_C1, q, inv[q]));
    fwd[q] = inv[q] = 0u;
    has[q] = 0;
  };
  for (size_t g = 0; g < F.op_words.size(); ++g) {
    const uint32_t w = F.op_words[g], k = op_kind(w), a = op_q0(w), b = op_q1(w);
    if (is_two_qubit(k)) {
      flush(a);
      flush(b);
      F.cl_words.push_back(w);
      back.push_back(w);  // CX and CZ are their own inverses
    } else {
      const uint32_t kinv = k == G_S ? (uint32_t)G_SDG : k == G_SDG ? (uint32_t)G_S : k;
      fwd[a] = c1_then(fwd[a], c1_of_gate(k));
      inv[a] = c1_then(c1_of_gate(kinv), inv[a]);  // the inverse run applies the last gate's inverse first
      has[a] = 1;
    }
  }
  for (uint32_t q = 0; q < m; ++q) flush(q);
  F.cl_back.assign(back.rbegin(), back.rend());
  layer_stream(F.cl_words, F.cl_layers, m);
  layer_stream(F.cl_back, F.cl_back_layers, m);
}

}  // namespace

int build_plan(uint32_t n, const HostOp *ops, size_t n_ops, const uint32_t *cut_q,
               const uint32_t *cut_after, size_t k, uint32_t max_nc, uint32_t max_cuts,
               PlanData &out, std::string &err) {
  if (n == 0 || n >= 16384) {
    err = "n_qubits must be in [1, 16383]";
    return CCUT_E_INVALID;
  }
  for (size_t i = 0; i < n_ops; ++i) {
    const HostOp &o = ops[i];
    if (o.kind > G_RZ) {
      err = "op " + std::to_string(i) + ": unknown gate kind";
      return CCUT_E_INVALID;
    }
    if (o.q0 >= n) {
      err = "op " + std::to_string(i) + ": qubit out of range";
      return CCUT_E_INVALID;
    }
    if (is_two_qubit(o.kind) && (o.q1 >= n || o.q1 == o.q0)) {
      err = "op " + std::to_string(i) + ": bad two-qubit operands";
      return CCUT_E_INVALID;
    }
  }
  std::set<std::pair<uint32_t, uint32_t>> seen;
  for (size_t c = 0; c < k; ++c) {
    if (cut_q[c] >= n || cut_after[c] >= n_ops) {
      err = "cut " + std::to_string(c) + ": out of range";
      return CCUT_E_INVALID;
    }
    const HostOp &o = ops[cut_after[c]];
    bool on = o.q0 == cut_q[c] || (is_two_qubit(o.kind) && o.q1 == cut_q[c]);
    if (!on) {
      err = "cut " + std::to_string(c) + ": op " + std::to_string(cut_after[c]) +
            " does not act on qubit " + std::to_string(cut_q[c]);
      return CCUT_E_INVALID;
    }
    if (!seen.insert({cut_q[c], cut_after[c]}).second) {
      err = "cut " + std::to_string(c) + ": duplicate";
      return CCUT_E_INVALID;
    }
  }
  if (k > max_cuts) {
    err = "k = " + std::to_string(k) + " cuts exceeds max_cuts = " + std::to_string(max_cuts);
    return CCUT_E_TOO_MANY_CUTS;
  }
  // position of each op along each of its wires
  std::vector<uint32_t> wire_len(n, 0);
  std::vector<uint32_t> pos0(n_ops), pos1(n_ops, 0);
  for (size_t i = 0; i < n_ops; ++i) {
    pos0[i] = wire_len[ops[i].q0]++;
    if (is_two_qubit(ops[i].kind)) pos1[i] = wire_len[ops[i].q1]++;
  }
  // cuts on each wire sorted by position; cut c separates segment s and s+1
  std::vector<std::vector<std::pair<uint32_t, uint32_t>>> wire_cuts(n);
  for (size_t c = 0; c < k; ++c) {
    const HostOp &o = ops[cut_after[c]];
    uint32_t p = (o.q0 == cut_q[c]) ? pos0[cut_after[c]] : pos1[cut_after[c]];
    wire_cuts[cut_q[c]].push_back({p, (uint32_t)c});
  }
  std::vector<uint32_t> seg_base(n + 1, 0);
  for (uint32_t q = 0; q < n; ++q) {
    std::sort(wire_cuts[q].begin(), wire_cuts[q].end());
    seg_base[q + 1] = seg_base[q] + (uint32_t)wire_cuts[q].size() + 1;
  }
  std::vector<uint32_t> cut_wire(k), cut_seg(k);
  for (uint32_t q = 0; q < n; ++q)
    for (size_t s = 0; s < wire_cuts[q].size(); ++s) {
      cut_wire[wire_cuts[q][s].second] = q;
      cut_seg[wire_cuts[q][s].second] = (uint32_t)s;
    }
  auto seg_of = [&](uint32_t q, uint32_t p) -> uint32_t {
    // segment index = number of cuts on the wire strictly before position p
    uint32_t s = 0;
    for (auto &wc : wire_cuts[q])
      if (wc.first < p) ++s;
    return s;
  };
  const uint32_t n_segs = seg_base[n];
  std::vector<uint32_t> op_seg0(n_ops), op_seg1(n_ops, 0);
  DSU dsu(n_segs);
  for (size_t i = 0; i < n_ops; ++i) {
    op_seg0[i] = seg_base[ops[i].q0] + seg_of(ops[i].q0, pos0[i]);
    if (is_two_qubit(ops[i].kind)) {
      op_seg1[i] = seg_base[ops[i].q1] + seg_of(ops[i].q1, pos1[i]);
      dsu.unite(op_seg0[i], op_seg1[i]);
    }
  }
  // components, ordered by their smallest (wire, segment), i.e. smallest global segment id
  std::map<uint32_t, std::vector<uint32_t>> comps;
  for (uint32_t s = 0; s < n_segs; ++s) comps[dsu.find(s)].push_back(s);
  std::vector<std::vector<uint32_t>> groups;
  for (auto &kv : comps) groups.push_back(kv.second);
  std::sort(groups.begin(), groups.end(),
            [](const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) { return a[0] < b[0]; });
  if (groups.size() > 255) {
    err = "more than 255 fragments";
    return CCUT_E_UNSUPPORTED;
  }
  std::vector<uint32_t> seg_wire(n_segs), seg_idx(n_segs);
  for (uint32_t q = 0; q < n; ++q)
    for (uint32_t s = seg_base[q]; s < seg_base[q + 1]; ++s) {
      seg_wire[s] = q;
      seg_idx[s] = s - seg_base[q];
    }
  std::vector<int32_t> seg_frag(n_segs), seg_local(n_segs);
  out = PlanData();
  out.n = n;
  out.k = (uint32_t)k;
  out.frags.resize(groups.size());
  for (size_t fi = 0; fi < groups.size(); ++fi) {
    Fragment &F = out.frags[fi];
    F.index = (uint32_t)fi;
    F.out_local.assign(n, -1);
    for (size_t j = 0; j < groups[fi].size(); ++j) {
      uint32_t s = groups[fi][j];  // ascending global id = ascending (wire, segment)
      seg_frag[s] = (int32_t)fi;
      seg_local[s] = (int32_t)j;
      F.wires.push_back(seg_wire[s]);
      F.segs.push_back(seg_idx[s]);
      if (s + 1 == seg_base[seg_wire[s] + 1]) F.out_local[seg_wire[s]] = (int32_t)j;
    }
  }
  for (size_t i = 0; i < n_ops; ++i) {
    Fragment &F = out.frags[seg_frag[op_seg0[i]]];
    uint32_t l0 = (uint32_t)seg_local[op_seg0[i]];
    uint32_t l1 = is_two_qubit(ops[i].kind) ? (uint32_t)seg_local[op_seg1[i]] : 0u;
    F.op_words.push_back(pack_op(ops[i].kind, l0, l1));
    F.op_theta.push_back(ops[i].theta);
    if (!is_clifford(ops[i].kind)) F.clifford = false;
  }
  for (size_t c = 0; c < k; ++c) {
    uint32_t up = seg_base[cut_wire[c]] + cut_seg[c];
    uint32_t down = up + 1;
    Fragment &Fu = out.frags[seg_frag[up]];
    Fu.axes.push_back({(uint32_t)c, 0u, (uint32_t)seg_local[up]});
    Fragment &Fd = out.frags[seg_frag[down]];
    Fd.axes.push_back({(uint32_t)c, 1u, (uint32_t)seg_local[down]});
  }
  for (Fragment &F : out.frags) {
    std::stable_sort(F.axes.begin(), F.axes.end(), [](const Axis &a, const Axis &b) {
      return a.cut != b.cut ? a.cut < b.cut : a.side < b.side;
    });
    if (F.axes.size() > (size_t)kMaxAxes) {
      err = "fragment " + std::to_string(F.index) + " has more than 16 cut axes";
      return CCUT_E_UNSUPPORTED;
    }
    uint64_t nv = 1;
    for (const Axis &a : F.axes) nv *= a.radix();
    if (nv > 0xFFFFFFFFull) {
      err = "fragment " + std::to_string(F.index) + " has more than 2^32 variants";
      return CCUT_E_UNSUPPORTED;
    }
    F.n_variants = nv;
    if (!F.clifford) {
      fuse_one_qubit_runs(F);
      if (F.m() <= (uint32_t)kMaxNcQubits) build_sv_program(F);
    } else {
      fuse_clifford_runs(F);
    }
    if (!F.clifford && F.m() > max_nc) {
      err = "non-Clifford fragment " + std::to_string(F.index) + " has " + std::to_string(F.m()) +
            " qubits > max_nc_qubits = " + std::to_string(max_nc);
      return CCUT_E_NC_TOO_WIDE;
    }
  }
  return CCUT_OK;
}

static FragRequest finish_request(const Fragment &f, std::vector<uint32_t> wanted_local,
                                  std::vector<uint32_t> wanted_user) {
  FragRequest r;
  std::set<uint32_t> meas(wanted_local.begin(), wanted_local.end());
  for (const Axis &a : f.axes)
    if (a.side == 0) meas.insert(a.local);
  r.meas.assign(meas.begin(), meas.end());
  std::map<uint32_t, uint32_t> pos;
  for (size_t j = 0; j < r.meas.size(); ++j) pos[r.meas[j]] = (uint32_t)j;
  std::vector<std::pair<uint32_t, uint32_t>> req;
  for (size_t i = 0; i < wanted_local.size(); ++i) req.push_back({pos[wanted_local[i]], wanted_user[i]});
  std::sort(req.begin(), req.end());
  for (auto &p : req) {
    r.req_pos.push_back(p.first);
    r.req_user.push_back(p.second);
  }
  for (const Axis &a : f.axes) r.axis_outpos.push_back(a.side == 0 ? (int32_t)pos[a.local] : -1);
  return r;
}

FragRequest marginal_request(const Fragment &f, const uint32_t *qubits, uint32_t nq) {
  std::vector<uint32_t> wl, wu;
  for (uint32_t i = 0; i < nq; ++i) {
    int32_t l = f.out_local[qubits[i]];
    if (l >= 0) {
      wl.push_back((uint32_t)l);
      wu.push_back(i);
    }
  }
  return finish_request(f, wl, wu);
}

FragRequest zstring_request(const Fragment &f, const std::vector<uint64_t> &anymask) {
  std::vector<uint32_t> wl, wu;
  for (uint32_t q = 0; q < (uint32_t)f.out_local.size(); ++q) {
    if (f.out_local[q] >= 0 && ((anymask[q >> 6] >> (q & 63)) & 1ull)) {
      wl.push_back((uint32_t)f.out_local[q]);
      wu.push_back(q);  // for Z strings the "user bit" is the circuit qubit
    }
  }
  return finish_request(f, wl, wu);
}

FragDev make_frag_dev(const Fragment &f, const FragRequest &r, uint64_t vid_base) {
  FragDev d{};
  d.m = f.m();
  d.n_ops = (uint32_t)(f.clifford ? f.cl_words.size() : f.sv_prog.size());
  d.n_axes = (uint32_t)f.axes.size();
  d.n_meas = (uint32_t)r.meas.size();
  d.n_req = (uint32_t)r.req_pos.size();
  d.clifford = f.clifford ? 1u : 0u;
  d.n_variants = f.n_variants;
  d.vid_base = vid_base;
  for (size_t j = 0; j < f.axes.size(); ++j) {
    d.axis_side[j] = f.axes[j].side;
    d.axis_local[j] = f.axes[j].local;
    d.axis_radix[j] = f.axes[j].radix();
    d.axis_cut[j] = f.axes[j].cut;
  }
  for (size_t j = 0; j < r.meas.size() && j < (size_t)kMaxMeas; ++j) d.meas[j] = (uint16_t)r.meas[j];
  return d;
}

}  // namespace ccut
