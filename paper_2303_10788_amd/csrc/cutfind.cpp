// Automatic cut placement (the circuit cutter of Sec. V-A): cut locations
// that isolate the non-Clifford operations in fragments no wider than a
// limit, with as few cuts as a greedy search finds (the recombination costs
// 4^k, Sec. III-B).  Host code only.
//
// A region is a set of wires, each with an interval of its ops (positions
// in the wire's op sequence).  It is closed when every two-qubit op inside
// an interval has its other operand's position inside that wire's interval
// too; a closed region is, after cutting at its interval ends, a fragment
// of its own.  Its cuts: one before the interval on every wire with earlier
// ops (a quantum input), one after it on every wire with later ops (a
// quantum output).
//
// Search: one region per non-Clifford op; then, while some move lowers the
// total cut count without exceeding the width limit, take the best one.
// Moves: merge two regions (the closure of their union, absorbing any
// region it overlaps), extend a region's interval on one wire to the
// wire's first or last op (closed again), or the composite cone moves below.  Each NC op needs at most two cuts
// on its own, so the result never exceeds 2 x (non-Clifford op count).
#include <algorithm>
#include <cstdint>
#include <map>
#include <vector>

#include "ccut.h"

namespace {

struct Circuit {
  uint32_t n;
  std::vector<ccut_op> ops;
  std::vector<std::vector<uint32_t>> wire_ops;    // per wire: op indices in order
  std::vector<std::map<uint32_t, uint32_t>> pos;  // per wire: op index -> position
};

bool two_qubit(uint32_t k) { return k == CCUT_CX || k == CCUT_CZ; }
bool non_clifford(uint32_t k) { return k == CCUT_T || k == CCUT_TDG || k == CCUT_RZ; }

using Region = std::map<uint32_t, std::pair<uint32_t, uint32_t>>;  // wire -> [lo, hi]

// Extend r until closed.
void close_region(const Circuit &C, Region &r) {
  std::vector<uint32_t> todo;
  for (auto &kv : r) todo.push_back(kv.first);
  std::map<uint32_t, std::pair<uint32_t, uint32_t>> done;  // wire -> interval already scanned
  while (!todo.empty()) {
    const uint32_t w = todo.back();
    todo.pop_back();
    const auto iv = r[w];
    auto it = done.find(w);
    const bool seen = it != done.end();
    for (uint32_t p = iv.first; p <= iv.second; ++p) {
      if (seen && p >= it->second.first && p <= it->second.second) continue;
      const ccut_op &o = C.ops[C.wire_ops[w][p]];
      if (!two_qubit(o.kind)) continue;
      const uint32_t u = o.q0 == w ? o.q1 : o.q0;
      const uint32_t pu = C.pos[u].at(C.wire_ops[w][p]);
      auto ru = r.find(u);
      if (ru == r.end()) {
        r[u] = {pu, pu};
        todo.push_back(u);
      } else if (pu < ru->second.first || pu > ru->second.second) {
        ru->second.first = std::min(ru->second.first, pu);
        ru->second.second = std::max(ru->second.second, pu);
        todo.push_back(u);
      }
    }
    done[w] = iv;
  }
}

uint32_t cost(const Circuit &C, const Region &r) {
  uint32_t k = 0;
  for (auto &kv : r) {
    k += kv.second.first > 0;
    k += kv.second.second + 1 < C.wire_ops[kv.first].size();
  }
  return k;
}

bool overlaps(const Region &a, const Region &b) {
  for (auto &kv : a) {
    auto it = b.find(kv.first);
    if (it != b.end() && kv.second.first <= it->second.second && it->second.first <= kv.second.second) return true;
  }
  return false;
}

Region unite(const Region &a, const Region &b) {
  Region r = a;
  for (auto &kv : b) {
    auto it = r.find(kv.first);
    if (it == r.end()) r[kv.first] = kv.second;
    else {
      it->second.first = std::min(it->second.first, kv.second.first);
      it->second.second = std::max(it->second.second, kv.second.second);
    }
  }
  return r;
}

// The closure of `seed` with every region it overlaps absorbed (repeatedly);
// `absorbed` lists the regions taken in.
Region absorb(const Circuit &C, Region seed, const std::vector<Region> &regs, std::vector<uint8_t> &absorbed) {
  for (bool grew = true; grew;) {
    grew = false;
    close_region(C, seed);
    for (size_t i = 0; i < regs.size(); ++i)
      if (!absorbed[i] && overlaps(seed, regs[i])) {
        seed = unite(seed, regs[i]);
        absorbed[i] = 1;
        grew = true;
      }
  }
  return seed;
}

// A composite move from region a: every wire of it taken to the circuit's
// start or end, closed, repeated until stable (the region's light cone that
// way); then single wires taken to the other end wherever that lowers the
// cut count.  This reaches block-shaped regions (a group of
// wires from the start, left through a few output cuts) that no single
// step reaches without first raising the count.
// dir 0: to the start, 1: to the end, 2: both (the region's whole
// connected component: no cuts at all when it fits).
Region cone_move(const Circuit &C, size_t a, int dir, const std::vector<Region> &regs, uint32_t max_width,
                 std::vector<uint8_t> &ab, bool &ok) {
  ok = false;
  const bool to_start = dir == 0;
  std::fill(ab.begin(), ab.end(), 0);
  ab[a] = 1;
  Region r = regs[a];
  for (;;) {
    Region s = r;
    for (auto &kv : s) {
      if (dir != 1) kv.second.first = 0;
      if (dir != 0) kv.second.second = (uint32_t)C.wire_ops[kv.first].size() - 1;
    }
    s = absorb(C, s, regs, ab);
    if (s.size() > max_width) return r;
    if (s == r) break;
    r = s;
  }
  if (dir == 2) {
    ok = true;
    return r;
  }
  auto net = [&](const Region &x, const std::vector<uint8_t> &abx) {
    long c = (long)cost(C, x);
    for (size_t i = 0; i < regs.size(); ++i)
      if (abx[i]) c -= (long)cost(C, regs[i]);
    return c;
  };
  for (bool improved = true; improved;) {
    improved = false;
    std::vector<uint32_t> wires;
    for (auto &kv : r) wires.push_back(kv.first);
    for (uint32_t w : wires) {
      Region s = r;
      if (to_start) s[w].second = (uint32_t)C.wire_ops[w].size() - 1;
      else s[w].first = 0;
      if (s == r) continue;
      std::vector<uint8_t> abs2 = ab;
      s = absorb(C, s, regs, abs2);
      if (s.size() <= max_width && net(s, abs2) < net(r, ab)) {
        r = s;
        ab = abs2;
        improved = true;
      }
    }
  }
  ok = true;
  return r;
}

}  // namespace

extern "C" ccut_status ccut_find_cuts(uint32_t n_qubits, const ccut_op *ops, size_t n_ops, uint32_t max_width,
                                      ccut_cut *cuts, size_t cap, size_t *k_out) {
  if (!k_out || (n_ops && !ops) || (cap && !cuts) || n_qubits == 0 || n_qubits >= 16384 || max_width == 0 ||
      n_ops > 0xFFFFFFFFull)
    return CCUT_E_INVALID;
  Circuit C;
  C.n = n_qubits;
  C.ops.assign(ops, ops + n_ops);
  C.wire_ops.assign(n_qubits, {});
  C.pos.assign(n_qubits, {});
  for (uint32_t i = 0; i < (uint32_t)n_ops; ++i) {
    const ccut_op &o = ops[i];
    if (o.kind > CCUT_RZ || o.q0 >= n_qubits) return CCUT_E_INVALID;
    if (two_qubit(o.kind) && (o.q1 >= n_qubits || o.q1 == o.q0)) return CCUT_E_INVALID;
    for (uint32_t w : {o.q0, o.q1}) {
      C.pos[w][i] = (uint32_t)C.wire_ops[w].size();
      C.wire_ops[w].push_back(i);
      if (!two_qubit(o.kind)) break;
    }
  }
  // one region per non-Clifford op (one wire wide)
  std::vector<Region> regs;
  for (uint32_t i = 0; i < (uint32_t)n_ops; ++i)
    if (non_clifford(ops[i].kind)) {
      const uint32_t p = C.pos[ops[i].q0][i];
      regs.push_back(Region{{ops[i].q0, {p, p}}});
    }
  auto width_ok = [&](const Region &r) { return r.size() <= max_width; };
  // best-improvement moves until none lowers the total cut count
  for (;;) {
    long best_gain = 0;
    Region best;
    std::vector<uint8_t> best_abs;
    auto consider = [&](const Region &seed, size_t self) {
      std::vector<uint8_t> ab(regs.size(), 0);
      ab[self] = 1;
      Region m = absorb(C, seed, regs, ab);
      if (!width_ok(m)) return;
      long before = 0;
      for (size_t i = 0; i < regs.size(); ++i)
        if (ab[i]) before += cost(C, regs[i]);
      const long gain = before - (long)cost(C, m);
      if (gain > best_gain) {
        best_gain = gain;
        best = m;
        best_abs = ab;
      }
    };
    auto take = [&](const Region &m, const std::vector<uint8_t> &ab) {
      long before = 0;
      for (size_t i = 0; i < regs.size(); ++i)
        if (ab[i]) before += cost(C, regs[i]);
      const long gain = before - (long)cost(C, m);
      if (gain > best_gain) {
        best_gain = gain;
        best = m;
        best_abs = ab;
      }
    };
    for (size_t a = 0; a < regs.size(); ++a) {
      for (int dir : {0, 1, 2}) {
        std::vector<uint8_t> ab(regs.size(), 0);
        bool ok = false;
        Region m = cone_move(C, a, dir, regs, max_width, ab, ok);
        if (ok) take(m, ab);
      }
      for (size_t b = a + 1; b < regs.size(); ++b) consider(unite(regs[a], regs[b]), a);
      for (auto &kv : regs[a]) {
        Region s = regs[a];
        s[kv.first].first = 0;
        consider(s, a);
        s = regs[a];
        s[kv.first].second = (uint32_t)C.wire_ops[kv.first].size() - 1;
        consider(s, a);
      }
    }
    if (best_gain <= 0) break;
    std::vector<Region> next;
    for (size_t i = 0; i < regs.size(); ++i)
      if (!best_abs[i]) next.push_back(regs[i]);
    next.push_back(best);
    regs.swap(next);
  }
  // initial single-op regions are closed and within any width >= 1; moves
  // keep regions closed and disjoint
  std::vector<ccut_cut> out;
  for (const Region &r : regs)
    for (auto &kv : r) {
      const auto &wo = C.wire_ops[kv.first];
      if (kv.second.first > 0) out.push_back({kv.first, wo[kv.second.first - 1]});
      if (kv.second.second + 1 < wo.size()) out.push_back({kv.first, wo[kv.second.second]});
    }
  std::sort(out.begin(), out.end(), [](const ccut_cut &x, const ccut_cut &y) {
    return x.after_op != y.after_op ? x.after_op < y.after_op : x.qubit < y.qubit;
  });
  // two regions meeting on a wire share the cut between them
  out.erase(std::unique(out.begin(), out.end(),
                        [](const ccut_cut &x, const ccut_cut &y) { return x.after_op == y.after_op && x.qubit == y.qubit; }),
            out.end());
  *k_out = out.size();
  for (size_t i = 0; i < out.size() && i < cap; ++i) cuts[i] = out[i];
  return out.size() <= cap ? CCUT_OK : CCUT_E_TOO_MANY_CUTS;
}
