// Shared definitions of the ccut device path: fragment descriptors read by
// every kernel, packed op words, and the host-side launchers of each kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccut {

constexpr int kMaxAxes = 16;   // cut axes incident to one fragment
constexpr int kMaxMeas = 64;   // measured qubits of one Clifford fragment (one u64 record)
constexpr int kMaxNcQubits = 12;  // state vector of 2^12 complex doubles = 64 KiB of LDS
constexpr int kMaxTableBits = 24;

enum GateKind : uint32_t {
  G_H = 0, G_S = 1, G_SDG = 2, G_X = 3, G_Y = 4, G_Z = 5, G_CX = 6, G_CZ = 7,
  G_T = 8, G_TDG = 9, G_RZ = 10
};

// op word: kind in bits 0-3, q0 in bits 4-17, q1 in bits 18-31 (local qubits < 16384)
__host__ __device__ inline uint32_t pack_op(uint32_t kind, uint32_t q0, uint32_t q1) {
  return (kind & 15u) | ((q0 & 0x3FFFu) << 4) | ((q1 & 0x3FFFu) << 18);
}
__host__ __device__ inline uint32_t op_kind(uint32_t w) { return w & 15u; }
__host__ __device__ inline uint32_t op_q0(uint32_t w) { return (w >> 4) & 0x3FFFu; }
__host__ __device__ inline uint32_t op_q1(uint32_t w) { return w >> 18; }

// One fragment under one request, as the kernels see it (device memory).
struct FragDev {
  uint32_t m;          // local qubits
  uint32_t n_ops;      // fragment gates (preparations and rotations are implied by the variant)
  uint32_t n_axes;
  uint32_t n_meas;     // measured set: requested circuit outputs + quantum outputs
  uint32_t n_req;      // requested circuit outputs among the measured set
  uint32_t clifford;
  uint64_t n_variants;
  uint64_t vid_base;   // (circuit << 40) | (fragment << 32)
  uint32_t axis_side[kMaxAxes];    // 0 quantum output (radix 3), 1 quantum input (radix 4)
  uint32_t axis_local[kMaxAxes];
  uint32_t axis_radix[kMaxAxes];
  uint32_t axis_cut[kMaxAxes];
  uint16_t meas[kMaxMeas];         // local qubit of measurement j (ascending)
  const uint32_t *ops;             // packed op words
  const double *theta;             // per op angle (RZ), may be null
};

// Per-variant affine sample model of a Clifford variant: a shot's outcome
// bits are x = x0 ^ (xor of G[:, a] over the random measurements a whose
// Philox bit is 1).  Layout per variant: [x0, randmask, Gcol[0..n_meas)].
__host__ __device__ inline uint32_t model_words(uint32_t n_meas) { return 2u + n_meas; }

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error.

hipError_t launch_tableau(const FragDev *d_frag, const FragDev &h_frag, uint64_t v0, uint64_t nv,
                          uint64_t *models, hipStream_t s);
hipError_t launch_sample_hist(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                              uint64_t seed, uint64_t vid0, uint32_t *partial, uint32_t nblk_x,
                              uint32_t quads_per_thread, uint64_t *records, hipStream_t s);
hipError_t launch_hist_reduce(const uint32_t *partial, uint64_t nv, uint32_t nblk_x, uint32_t bins,
                              uint64_t shots, double *dist, hipStream_t s);
hipError_t launch_exact_tables(const uint64_t *models, uint32_t n_meas, uint64_t nv, double *dist,
                               hipStream_t s);
hipError_t launch_sv(const FragDev *d_frag, const FragDev &h_frag, uint64_t v0, uint64_t nv,
                     double *dist, hipStream_t s);
hipError_t launch_parity_exact(const uint64_t *models, uint32_t n_meas, uint64_t nv,
                               const uint64_t *ext_masks, uint32_t n_ext, double *E, hipStream_t s);
hipError_t launch_parity_sampled(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                                 uint64_t seed, uint64_t vid0, const uint64_t *ext_masks,
                                 uint32_t n_ext, uint32_t *odd_counts, hipStream_t s);
hipError_t launch_parity_finish(const uint32_t *odd_counts, uint64_t n, uint64_t shots, double *E,
                                hipStream_t s);
hipError_t launch_dist_parity(const double *dist, uint32_t n_meas, uint64_t nv,
                              const uint64_t *ext_masks, uint32_t n_ext, double *E, hipStream_t s);
// One Pauli-basis pass over cut axis j: mode 0 = quantum input (4 -> 4),
// mode 1 = quantum output on outcome distributions (basis x outcome -> 4),
// mode 2 = quantum output on parity tables (basis x J-bit -> 4).
hipError_t launch_transform_pass(const double *in, double *out, uint64_t outer, uint64_t inner_digits,
                                 uint64_t xsize_in, uint64_t lo, int mode, hipStream_t s);

struct RecombFrag {
  const double *T;          // T_f[p_f][row], row count `rows`
  uint32_t n_axes;
  uint32_t rows;
  uint32_t n_req;
  uint32_t axis_cut[kMaxAxes];
  uint32_t req_user[32];    // output bit of each requested row bit
};
constexpr int kMaxFrags = 64;
struct RecombArgs {
  uint32_t n_frags;
  uint32_t k;
  RecombFrag f[kMaxFrags];
};
hipError_t launch_recombine_fp64(const RecombArgs *d_args, uint32_t nq, double *out, hipStream_t s);
hipError_t launch_zrecombine_fp64(const RecombArgs *d_args, uint32_t n_strings, double *out, hipStream_t s);

}  // namespace ccut
