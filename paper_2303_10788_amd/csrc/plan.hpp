// Host-side planning: validate a circuit and cut list, split cut wires into
// segments, form fragments (connected components of segments joined by
// two-qubit gates), tag Clifford fragments, number variants, and derive the
// per-fragment view of a marginal or Z-string request.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "common.hpp"

namespace ccut {

struct HostOp {
  uint32_t kind, q0, q1;
  double theta;
};

struct Axis {
  uint32_t cut;    // index in the cut list
  uint32_t side;   // 0 quantum output (upstream of the cut), 1 quantum input
  uint32_t local;  // fragment-local qubit
  uint32_t radix() const { return side == 0 ? 3u : 4u; }
};

struct Fragment {
  uint32_t index = 0;
  std::vector<uint32_t> wires, segs;        // local qubit i = (wires[i], segs[i])
  std::vector<uint32_t> op_words;           // packed local ops, in circuit order
  std::vector<double> op_theta;
  // Clifford fragments: runs of one-qubit gates on a qubit fused into one
  // G_C1 word (cl_words, circuit order), and the inverse stream for the
  // Heisenberg carry-back (cl_back: last gate first, each gate inverted)
  std::vector<uint32_t> cl_words, cl_back;
  // both streams are ordered by ASAP layer; layer L of a stream spans
  // words [layers[L], layers[L + 1])
  std::vector<uint32_t> cl_layers, cl_back_layers;
  // non-Clifford fragments: the same ops with runs of one-qubit gates on a
  // qubit fused into one 2x2 unitary (G_U2) for the state-vector kernel
  std::vector<uint32_t> sv_words;
  std::vector<double> sv_mats;              // 8 doubles per sv word
  // the same stream laid out for the state-vector kernel (SV_* words, 8
  // doubles per word)
  std::vector<uint32_t> sv_prog;
  std::vector<double> sv_prog_mats;
  bool clifford = true;
  std::vector<Axis> axes;
  std::vector<int32_t> out_local;           // per wire: local qubit if this fragment ends the wire, else -1
  uint64_t n_variants = 1;
  uint32_t m() const { return (uint32_t)wires.size(); }
};

struct PlanData {
  uint32_t n = 0;
  uint32_t k = 0;
  std::vector<Fragment> frags;
};

// Returns 0 on success, else a ccut_status code with `err` filled.
int build_plan(uint32_t n, const HostOp *ops, size_t n_ops, const uint32_t *cut_q,
               const uint32_t *cut_after, size_t k, uint32_t max_nc, uint32_t max_cuts,
               PlanData &out, std::string &err);

// Per-fragment view of a request.
struct FragRequest {
  std::vector<uint32_t> meas;      // measured local qubits, ascending
  std::vector<uint32_t> req_pos;   // positions in meas of the requested circuit outputs
  std::vector<uint32_t> req_user;  // their output bit (index in the user's qubit list)
  std::vector<int32_t> axis_outpos;  // per axis: position in meas (outputs), -1 for inputs
};

FragRequest marginal_request(const Fragment &f, const uint32_t *qubits, uint32_t nq);
// Z strings: every circuit output of the fragment that occurs in any mask,
// plus its quantum outputs.  `anymask` has ceil(n/64) words.
FragRequest zstring_request(const Fragment &f, const std::vector<uint64_t> &anymask);

FragDev make_frag_dev(const Fragment &f, const FragRequest &r, uint64_t vid_base);

}  // namespace ccut
