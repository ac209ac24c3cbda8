// Shared definitions of the ccut device path: fragment descriptors read by
// every kernel, packed op words, and the host-side launchers of each kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccut {

constexpr int kMaxAxes = 16;   // cut axes incident to one fragment
constexpr int kMaxMeas = 64;   // measured qubits of one Clifford fragment (one u64 record)
constexpr int kMaxNcQubits = 12;  // state vector of 2^12 complex doubles = 64 KiB of LDS

// State-vector programs.  A non-Clifford fragment's state of 2^m amplitudes
// is spread over registers: amplitude index bits [0, RB) select one of a
// thread's 2^RB registers, the next min(m, 6) bits the lane of a wave and
// the top WB bits the wave.  A program maps each logical qubit to one of
// these bit positions; ops whose matrix mixes amplitudes (a general 2x2 or
// a CX target) act on register or lane positions only, so they need no
// barrier; diagonal ops, CZ and CX controls act anywhere.  SV_SWAP exchanges
// a register or lane position with a wave position through LDS.
enum : uint32_t {
  SV_U2 = 0,    // general 2x2 unitary on position a (register or lane), matrix in mats
  SV_DIAG = 1,  // diagonal unitary on position a (any): diag(m00, m11)
  SV_CX = 2,    // control position a (any), target position b (register or lane)
  SV_CZ = 3,    // positions a, b (any)
  SV_SWAP = 4,  // exchange positions a (register or lane) and b (wave)
  SV_END = 5,   // final layout: bits 4q..4q+3 of the first matrix word = position of qubit q
};
struct SvShape {
  uint32_t rb, lb, wb;  // register, lane and wave bits
};
// Up to 4 amplitudes per thread (more spill registers): one wave up to 8
// qubits (register bits first, so ops on the two lowest positions need no
// exchange), and from 9 qubits on the state spreads over 2^(m - 8) waves,
// up to 16 (1024 threads).  Every state of up to 8 qubits (from 2) has the
// same shape, so a batch runs them in one launch.
__host__ __device__ inline SvShape sv_shape(uint32_t m) {
  if (m <= 8) {
    const uint32_t rb = m < 2 ? m : 2u;
    return {rb, m - rb, 0u};
  }
  return {2u, 6u, m - 8};
}
constexpr int kMaxTableBits = 24;

enum GateKind : uint32_t {
  G_H = 0, G_S = 1, G_SDG = 2, G_X = 3, G_Y = 4, G_Z = 5, G_CX = 6, G_CZ = 7,
  G_T = 8, G_TDG = 9, G_RZ = 10,
  G_U2 = 11,   // fused one-qubit unitary (state-vector path only), matrix in FragDev::mats
  G_C1 = 12,   // fused one-qubit Clifford (tableau paths), parameters in the q1 field
  G_NOP = 15   // padding of op arrays to a multiple of 4 words
};

// op word: kind in bits 0-3, q0 in bits 4-17, q1 in bits 18-31 (local qubits < 16384)
__host__ __device__ inline uint32_t pack_op(uint32_t kind, uint32_t q0, uint32_t q1) {
  return (kind & 15u) | ((q0 & 0x3FFFu) << 4) | ((q1 & 0x3FFFu) << 18);
}
__host__ __device__ inline uint32_t op_kind(uint32_t w) { return w & 15u; }
__host__ __device__ inline uint32_t op_q0(uint32_t w) { return (w >> 4) & 0x3FFFu; }
__host__ __device__ inline uint32_t op_q1(uint32_t w) { return w >> 18; }

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of
// (c0..c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
// key bumped by the Weyl constants between rounds.
struct U4 {
  uint32_t w[4];
};

__device__ inline U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                              uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return U4{{c0, c1, c2, c3}};
}

// One-qubit Clifford action on a Pauli row's bits (x, z) at its qubit and
// on the row's sign c (the tableau update rule P -> G P G^dag): new
// (x, z) = M (x, z) over GF(2) and c ^= alpha x ^ beta z ^ gamma x z, both
// from the bits before the gate.  Any run of one-qubit Cliffords composes
// to this form.  Encoded in the q1 field of a G_C1 word: bits 0-3 hold
// M xor I (m00, m01, m10, m11), bits 4-6 alpha, beta, gamma, so an all-zero
// field (also every G_NOP word) is the identity.
struct C1Map {
  uint32_t m00, m01, m10, m11, al, be, ga;
};
__host__ __device__ inline C1Map c1_decode(uint32_t p) {
  return C1Map{(p & 1u) ^ 1u, (p >> 1) & 1u, (p >> 2) & 1u, ((p >> 3) & 1u) ^ 1u, (p >> 4) & 1u, (p >> 5) & 1u,
               (p >> 6) & 1u};
}
__host__ __device__ inline uint32_t c1_encode(const C1Map &c) {
  return (c.m00 ^ 1u) | (c.m01 << 1) | (c.m10 << 2) | ((c.m11 ^ 1u) << 3) | (c.al << 4) | (c.be << 5) | (c.ga << 6);
}
// the single gates: H swaps x and z (c ^= x z); S and S^dag map z -> x ^ z
// (c ^= x z, resp. x (1 ^ z)); X, Y, Z flip c by z, x ^ z, x
__host__ __device__ inline uint32_t c1_of_gate(uint32_t kind) {
  switch (kind) {
    case G_H: return c1_encode(C1Map{0, 1, 1, 0, 0, 0, 1});
    case G_S: return c1_encode(C1Map{1, 0, 1, 1, 0, 0, 1});
    case G_SDG: return c1_encode(C1Map{1, 0, 1, 1, 1, 0, 1});
    case G_X: return c1_encode(C1Map{1, 0, 0, 1, 0, 1, 0});
    case G_Y: return c1_encode(C1Map{1, 0, 0, 1, 1, 1, 0});
    case G_Z: return c1_encode(C1Map{1, 0, 0, 1, 1, 0, 0});
    default: return 0u;
  }
}
// the map of "first a, then b"
__host__ __device__ inline uint32_t c1_then(uint32_t pa, uint32_t pb) {
  const C1Map A = c1_decode(pa), B = c1_decode(pb);
  C1Map C;
  C.m00 = (B.m00 & A.m00) ^ (B.m01 & A.m10);
  C.m01 = (B.m00 & A.m01) ^ (B.m01 & A.m11);
  C.m10 = (B.m10 & A.m00) ^ (B.m11 & A.m10);
  C.m11 = (B.m10 & A.m01) ^ (B.m11 & A.m11);
  // B's sign form evaluated on A's output: x1 = m00 x ^ m01 z, z1 = m10 x ^ m11 z,
  // x1 z1 = m00 m10 x ^ m01 m11 z ^ det(A) x z (bits: x^2 = x, z^2 = z)
  C.al = A.al ^ (B.al & A.m00) ^ (B.be & A.m10) ^ (B.ga & A.m00 & A.m10);
  C.be = A.be ^ (B.al & A.m01) ^ (B.be & A.m11) ^ (B.ga & A.m01 & A.m11);
  C.ga = A.ga ^ (B.ga & ((A.m00 & A.m11) ^ (A.m01 & A.m10)));
  return c1_encode(C);
}

// Global-address-space views: loads through them with a wave-uniform index
// compile to scalar (SMEM) loads, so op decoding stays in SGPRs.
typedef __attribute__((address_space(1))) const uint32_t g_u32;
typedef __attribute__((address_space(1))) const double g_double;

// Four op words starting at word 4*g4 (a uniform index: one scalar load).
__device__ inline uint4 load_ops4(const uint32_t *ops, uint32_t g4) {
  const g_u32 *p = (const g_u32 *)ops + 4 * g4;
  return make_uint4(p[0], p[1], p[2], p[3]);
}

// Sixteen op words starting at word 16*g16: one wait per sixteen gates
// (op arrays are padded with G_NOP to a multiple of 16 words).
struct Ops16 {
  uint32_t w[16];
};
__device__ inline Ops16 load_ops16(const uint32_t *ops, uint32_t g16) {
  const g_u32 *p = (const g_u32 *)ops + 16 * g16;
  Ops16 o;
#pragma unroll
  for (int i = 0; i < 16; ++i) o.w[i] = p[i];
  return o;
}

// One fragment under one request, as the kernels see it (passed by value in
// the kernel-argument segment, so every field read is a scalar load).
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
  const uint32_t *ops;             // packed op words, padded with G_NOP to a multiple of 16
  const double *mats;              // per op 2x2 complex matrix (re00 im00 re01 im01 re10 im10 re11 im11), G_U2 only
  // Clifford streams come in ASAP layers of ops on disjoint qubits (layer L
  // is ops[layers[L] .. layers[L + 1])); reordering commuting ops changes
  // no row and no sign
  const uint32_t *layers;
  uint32_t n_layers;
  uint32_t pad_;
};

// Per-variant affine sample model of a Clifford variant: a shot's outcome
// bits are x = x0 ^ (xor of G[:, a] over the random measurements a whose
// Philox bit is 1).  Layout per variant: [x0, randmask, Gcol[0..n_meas)].
// Words of one outcome vector in a model: 1 up to 64 measurements, else
// the power of two at or above ceil(n / 64) (at most 16: kMaxMeasWide).
// Model: x0, randmask, then G[a] for each measurement a, each that many
// words.
constexpr int kMaxMeasWide = 1024;
__host__ __device__ inline uint32_t model_mw(uint32_t n_meas) {
  const uint32_t w = (n_meas + 63) / 64;
  return w <= 1 ? 1u : w <= 2 ? 2u : w <= 4 ? 4u : w <= 8 ? 8u : 16u;
}
__host__ __device__ inline uint32_t model_words(uint32_t n_meas) { return model_mw(n_meas) * (2u + n_meas); }

// One unit of the batched model launch: variant `variant` of descriptor
// `desc`, its model written at word offset `model_off`.
struct BatchItem {
  uint32_t desc;
  uint32_t pad;
  uint64_t variant;
  uint64_t model_off;
  uint64_t base_off;  // word offset of the fragment's carried-back measured rows
};

// One fragment's sampled outcome tables in a batched launch: variants
// [0, nv) of `models`, nblk shot blocks per variant (qpt quads per thread),
// counts in `partial` (per block when n_meas <= 14 or sliced, else per
// variant, zeroed beforehand), tables in `dist`.  wg0 / rb0: the job's first workgroup of
// the sampling launch and of the reduction launch (4096 entries each).
struct SampleJob {
  const uint64_t *models;
  uint32_t *partial;
  double *dist;
  uint16_t *cnt16;  // when set: the tables as 16-bit shot counts (shots < 2^16) instead of dist
  uint64_t shots, seed, vid0, nv;
  uint64_t wg0, rb0;
  uint32_t n_meas, nblk, qpt;
  uint32_t nslice;  // > 1: n_meas > kLdsHistBits counted in LDS slices of 2^kLdsHistBits bins
};

// Sampling LDS: the shot xor's byte tables (256 u64 per 8 measurement
// indices) and the workgroup's histogram of up to 2^kLdsHistBits bins,
// 16-bit counts packed two to a 32-bit word.  A workgroup counts at most
// kMaxUnitShots shots (at most kMaxUnitQpt quads per thread), so no count
// carries into its neighbour.  Wider outcome tables are counted in
// 2^kLdsHistBits-bin slices (up to kMaxSliceBits more bits), each slice
// replaying the shots.
constexpr uint32_t kLdsHistBits = 16;
constexpr uint32_t kMaxSliceBits = 3;
constexpr uint32_t kSampleThreads = 256;  // threads of a sampling workgroup (512: no faster)
constexpr uint32_t kMaxUnitQpt = 63;      // 63 quads x 256 threads x 4 shots = 64512 < 2^16
static_assert(kMaxUnitQpt * kSampleThreads * 4 < 65536, "16-bit LDS counts");
__host__ __device__ inline uint32_t sample_tab_groups(uint32_t n_meas) { return (n_meas + 7) / 8; }
inline size_t sample_lds_bytes(uint32_t n_meas, bool hist, bool sliced = false) {
  const size_t tab = (size_t)sample_tab_groups(n_meas) * 256 * 8;
  if (!hist) return tab;
  const uint32_t lb = sliced ? kLdsHistBits : n_meas;
  if (lb > kLdsHistBits) return tab;
  return tab + 4 * (((size_t(1) << lb) + 1) / 2);
}
constexpr size_t kSampleLdsMax = 8 * 256 * 8 + (size_t(2) << kLdsHistBits);

// One non-Clifford fragment in a batched state-vector launch: descriptor
// descs[desc], tables in dist, wg0 = its first workgroup.
// One fragment's pass of a batched state-vector launch: mode 0 runs every
// preparation combination in full (fragments without quantum inputs),
// mode 1 evolves the computational-basis inputs into `states`, mode 2
// combines them into the preparation combinations' tables.
struct SvJob {
  uint32_t desc, split;
  uint64_t wg0;
  double *dist;
  uint32_t mode, pad_;
  double *states;  // [2^n_in][2^m] complex amplitudes (modes 1 and 2)
};

// The job whose range [start, next start) holds idx (starts ascending, first 0).
template <class J, class F>
__device__ inline uint32_t find_job(const J *jobs, uint32_t n, uint64_t idx, F start) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (start(jobs[mid]) <= idx) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The dispatcher hands consecutive workgroups of a launch to the chip's 8
// XCDs in turn, and each XCD has an L2 of its own.  xcd_block renumbers
// workgroup `bid` of `n` so that each XCD runs one contiguous range of
// logical blocks: neighbouring tiles, which share cache lines, then meet in
// one L2 instead of being fetched from HBM once per XCD.  A bijection of
// [0, n) for any n.
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t n) {
  const uint32_t x = bid % kXcds, local = bid / kXcds, per = n / kXcds, rem = n % kXcds;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error.

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s);
hipError_t launch_sample_hist(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                              uint64_t seed, uint64_t vid0, uint32_t *partial, uint32_t nblk_x,
                              uint32_t quads_per_thread, uint64_t *records, hipStream_t s,
                              const uint8_t *vmask = nullptr);
hipError_t launch_hist_reduce(const uint32_t *partial, uint64_t nv, uint32_t nblk_x, uint32_t bins,
                              uint64_t shots, double *dist, hipStream_t s, uint16_t *cnt16 = nullptr);
hipError_t launch_exact_tables(const uint64_t *models, uint32_t n_meas, uint64_t nv, double *dist,
                               hipStream_t s);
// prog: the fragment's state-vector program (words + 8 doubles per word)
// states: scratch of sv_states_bytes(frag) (may be NULL when it is 0).
hipError_t launch_sv(const FragDev &frag, double *dist, void *states, hipStream_t s);
uint32_t sv_inputs(const FragDev &h);
size_t sv_states_bytes(const FragDev &h);
// Launch shape of one pass (0 full, 1 evolve, 2 combine) of a fragment.
void sv_pass_shape(const FragDev &h, uint32_t pass, uint64_t &n_wg, uint32_t &block, size_t &lds, bool &split);
// State-vector launch shape of a fragment: workgroups, threads, LDS bytes,
// whether basis combinations get workgroups of their own.
void sv_launch_shape(const FragDev &h, uint64_t &n_wg, uint32_t &block, size_t &lds, bool &split);
// Many non-Clifford fragments of one shape (same m class: register bits and
// waves) in one launch; lds = the largest of theirs.
hipError_t launch_sv_batch(const FragDev *descs, const SvJob *jobs, uint32_t n_jobs, uint64_t total_wg, uint32_t m,
                           size_t lds, hipStream_t s);
// Batched sampling over jobs (see SampleJob; wg0 numbers the units of this
// launch's jobs from 0); lds = the largest sample_lds_bytes among them.  The
// reduction runs over all jobs of a batch (rb0 numbering) in one launch.
hipError_t launch_sample_batch(const SampleJob *jobs, uint32_t n_jobs, uint64_t total_units, size_t lds,
                               hipStream_t s);
hipError_t launch_hist_reduce_batch(const SampleJob *jobs, uint32_t n_jobs, uint64_t total_reduce_blocks,
                                    hipStream_t s);
hipError_t launch_parity_exact(const uint64_t *models, uint32_t n_meas, uint64_t nv,
                               const uint64_t *ext_masks, uint32_t n_ext, double *E, hipStream_t s);
hipError_t launch_parity_sampled(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                                 uint64_t seed, uint64_t vid0, const uint64_t *ext_masks,
                                 uint32_t n_ext, uint32_t *odd_counts, hipStream_t s);
hipError_t launch_parity_finish(const uint32_t *odd_counts, uint64_t n, uint64_t shots, bool settle, double *E,
                                hipStream_t s);
// The same over more than 64 measurements (wide models, model_mw words per
// vector): ext_masks [n_ext][model_mw], odd_counts zeroed by the caller;
// shot records [nv][shots][ceil(n_meas / 64)].
hipError_t launch_parity_exact_wide(const uint64_t *models, uint32_t n_meas, uint64_t nv, const uint64_t *ext_masks,
                                    uint32_t n_ext, double *E, hipStream_t s);
hipError_t launch_parity_sampled_wide(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                                      uint64_t seed, uint64_t vid0, const uint64_t *ext_masks, uint32_t n_ext,
                                      uint32_t *odd_counts, hipStream_t s);
hipError_t launch_records_wide(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots, uint64_t seed,
                               uint64_t vid0, uint64_t *records, hipStream_t s);
hipError_t launch_dist_parity(const double *dist, uint32_t n_meas, uint64_t nv,
                              const uint64_t *ext_masks, uint32_t n_ext, double *E, hipStream_t s);
// One Pauli-basis pass over cut axis j: mode 0 = quantum input (4 -> 4),
// mode 1 = quantum output on outcome distributions (basis x outcome -> 4),
// mode 2 = quantum output on parity tables (basis x J-bit -> 4).
// All Pauli-basis passes of one fragment in one launch: out[P][x_out] is
// the sum over the per-axis coefficient terms (input axis: I = p0 + p1,
// X = 2p+ - p0 - p1, Y = 2p+i - p0 - p1, Z = p0 - p1; output axis, per
// outcome bit b of its basis: I = b0 + b1 (Z basis), X, Y, Z = b0 - b1;
// Z-string selection: I picks b0 of Z, X/Y/Z pick b1 of their basis).
// Digit j of the variant index (axis 0 fastest) has radix rad[j]; P has four
// values per axis, axis 0 fastest; x is the fastest index.
struct TransformAll {
  uint32_t n_axes;
  uint32_t mode[kMaxAxes];  // 0 quantum input, 1 output (outcome bit), 2 output (string selection)
  uint32_t rad[kMaxAxes];
  uint32_t pos[kMaxAxes];   // mode 1: outcome bit position in the input's x
  uint64_t x_in, x_out;
  uint64_t n_strings;       // mode 2: x_in = J * n_strings + x_out, bit t of J = t-th output axis
};
hipError_t launch_transform_all(const TransformAll &a, const double *in, double *out, hipStream_t s);

// Pauli transform of one fragment's variant tables, tiled through LDS: the
// per-axis passes (same operations, same axis order as the pass kernel) on
// a tile of 2^t output entries at a time, all axes in one launch.  The
// variant data of a tile (v_count x 2^lbits doubles, the outcome bits of the
// output axes inside) must fit kTileElems.  Layout of a tile's x: the x_in
// bits below thr, then the outcome bits at x_in positions hpos[0..nh).
constexpr int kMaxTileAxes = 8;
constexpr uint32_t kTileElems = 4096, kTileMaxT = 8;
struct TileJob {
  const double *in;
  double *out;
  const uint16_t *in16;  // when set: the variant data as 16-bit shot counts, value = count / shots
  double shots;
  uint64_t x_in, x_out;
  uint64_t wg0;                 // first workgroup of the job in a batched launch
  uint32_t tiles;               // x_out >> t
  uint32_t n_axes, v_count, t, thr, nh, lbits;
  uint32_t fold;                // axes (bit j) rewritten into the downstream preparation basis (launch_fold's map)
  uint32_t rad[kMaxTileAxes];   // 4 quantum input, 3 quantum output
  uint32_t lpos[kMaxTileAxes];  // output axis: its outcome bit's position in the tile's x
  uint32_t hpos[kMaxTileAxes];  // x_in positions of the outcome bits at or above thr, ascending
  uint32_t xpos[kTileMaxT];     // the t positions below thr that carry the tile's x_out bits, ascending
  uint32_t rmag[kMaxTileAxes];  // floor(2^32 / R_j) + 1, R_j the product of the radices below axis j (0: R_j = 1)
};
hipError_t launch_transform_tiled(const TileJob *d_jobs, uint32_t n_jobs, uint64_t total_wg, hipStream_t s);

hipError_t launch_transform_pass(const double *in, double *out, uint64_t outer, uint64_t inner_digits,
                                 uint64_t xsize_in, uint64_t lo, int mode, hipStream_t s);

// Exact Pauli-basis tensor of a Clifford fragment without enumerating
// variants (Heisenberg picture); see k_heis.hip for the row layout.
// Rows carried through F.ops (F.n_ops words), column-sliced (k_heis.hip):
// rows_in null starts from the identity tableau (X_r for r < m, then
// Z_{r-m}); rows are (x[W], z[W], sign) u64 each.
hipError_t launch_rows(const FragDev &F, uint32_t W, const uint64_t *in, uint64_t *out, uint32_t n_rows,
                       hipStream_t s);
// One fragment's carry-back in a batched launch: n_rows rows of width W
// words per half at in + in_off, carried through the descriptor's stream
// into out + out_off.
struct CarryJob {
  uint32_t desc, W, n_rows, pad_;
  uint64_t in_off, out_off;
};
hipError_t launch_carry_batch(const FragDev *descs, const CarryJob *jobs, uint32_t n_jobs, uint32_t max_m,
                              uint32_t max_rows, const uint64_t *in, uint64_t *out, hipStream_t s);
// Affine sample models from carried-back measured Paulis (one wave per
// variant): rows as built by measured_rows on the host, W words per half.
hipError_t launch_affine(const FragDev &F, uint32_t W, const uint64_t *rows, uint64_t v0, uint64_t nv,
                         uint64_t *models, hipStream_t s, const uint8_t *vmask = nullptr);
// More than 64 measurements (up to kMaxMeasWide): one workgroup per
// variant; meas_axis[j] = the axis of measurement j if it is a quantum
// output, else -1; row_of[j] = its first row in `rows`.
hipError_t launch_affine_wide(const FragDev &F, uint32_t W, const int8_t *meas_axis, const uint16_t *row_of,
                              uint32_t n_meas, const uint64_t *rows, uint64_t v0, uint64_t nv, uint64_t *models,
                              hipStream_t s);
// desc_w[d]: row width of descriptor d; BatchItem::base_off: word offset of
// the item's fragment rows; block threads (a multiple of 64), grid blocks.
hipError_t launch_affine_batch(const FragDev *descs, const uint32_t *desc_w, const BatchItem *items, uint32_t n_items,
                               const uint64_t *rows, uint64_t *models, uint32_t block, uint32_t grid, hipStream_t s);
hipError_t launch_heisenberg(const FragDev &F, uint32_t W, uint32_t n_in, uint32_t n_out, uint32_t r,
                             uint32_t n_str, const uint64_t *cin_mask, const uint64_t *rows_in, uint64_t *rows_out,
                             uint32_t n_rows, double *tau, hipStream_t s);

// A fragment tensor to be rewritten along cut axes `mask` (bit j = axis j)
// into the preparation basis of the fragments downstream (launch_fold).
struct FoldJob {
  double *T;
  uint64_t rows;
  uint32_t n_axes, mask;
};
hipError_t launch_fold(const FoldJob *d_jobs, uint32_t n_jobs, hipStream_t s);

// Maximum-likelihood correction of one fragment's variant tables (in
// place): n_out (1 or 2) quantum outputs, n_in inputs.
constexpr uint32_t kMlMaxOut = 2;
struct MlJob {
  double *dist;       // [n_variants][row_len] tables, corrected in place
  double *eig;        // scratch: [n_prep][nx][2^n_out] eigenvalues
  double *tau;        // scratch: [n_prep] simplex shifts
  uint64_t nx;        // 2^n_req outcomes of the requested outputs
  uint64_t row_len;   // 2^(measured bits)
  uint32_t n_prep;    // 4^n_in
  uint32_t n_out, n_in, n_req;
  uint32_t opos[kMlMaxOut];     // outcome bit of each quantum output (axis order)
  uint32_t ostride[kMlMaxOut];  // its variant-index stride
  uint32_t istride[kMaxAxes];   // variant-index stride of each quantum input (axis order)
  uint32_t xpos[32];            // outcome bit of each requested output
};
hipError_t launch_ml_correct(const MlJob &h, const MlJob *d_job, hipStream_t s);

struct RecombFrag {
  const double *T;          // T_f[p_f][row], row count `rows`
  uint32_t cnt16;           // 1: T holds 16-bit shot counts, the value is count / shots
  uint32_t pad_;
  double shots;
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
  uint32_t lo_parts;  // fp32 modes: 1 = hi/lo split operands (three products), 0 = fp32 operands
  RecombFrag f[kMaxFrags];
};
hipError_t launch_recombine_fp64(const RecombArgs *d_args, uint32_t n_frags, uint32_t nq, double *out,
                                 hipStream_t s);
// Batched plain fp64 recombination (at most 8 fragments per job): job j's
// workgroups [wg0, next wg0) cover its 2^nq outputs, 128 per workgroup.
struct RcJob {
  const RecombArgs *args;
  double *const *out;  // slot holding the output address (read when the job runs)
  uint64_t wg0;
  uint32_t nq, pad_;
};
hipError_t launch_recombine_batch(const RcJob *d_jobs, uint32_t n_jobs, uint64_t total_wg, hipStream_t s);
// The plain fp64 sum over a term list (ascending cut terms; at most 8
// fragments): the same operations as the full sum without its zero terms.
hipError_t launch_recombine_terms(const RecombArgs *d_args, uint32_t nq, const uint64_t *terms, uint64_t n_terms,
                                  double *out, hipStream_t s);
// Sparse support of a contraction: nz[off_f + p] = 1 if column p of
// fragment f's tensor has a nonzero entry; then the cut terms P with every
// fragment's column nonzero, ascending, into terms[0 .. count) and the
// count into *count (device).  pos: K words, scratch: scan_scratch_words(K).
struct SupportArgs {
  uint64_t off[kMaxFrags];
};
hipError_t launch_colnz(const double *T, uint32_t rows, uint64_t cols, uint8_t *nz, hipStream_t s);

// One result vector to copy: n doubles from src to dst (device memory).
struct OutCopy {
  const double *src;
  double *dst;
  uint64_t n;
};
// All copies in one launch (at most 65535 of them; max_n = the longest n).
hipError_t launch_gather_f64(const OutCopy *d_jobs, uint32_t n_jobs, uint64_t max_n, hipStream_t s);
hipError_t launch_support_terms(const RecombArgs *d_args, const SupportArgs &sa, const uint8_t *nz, uint64_t K,
                                uint64_t *pos, uint64_t *scratch, uint64_t *terms, hipStream_t s);
constexpr uint32_t kRcChunkOut = 128;  // outputs per workgroup of the plain recombination
// Z strings: fp64 products and sum, or (fp32 = true) fp32 products summed
// in fp32 over chunks of 32 terms and in fp64 across chunks.
uint32_t zrecombine_splits(uint32_t k, uint32_t n_strings);
hipError_t launch_zrecombine(const RecombArgs *d_args, uint32_t n_frags, uint32_t k, uint32_t n_strings, bool fp32,
                             double *partial, uint32_t splits, double *out, hipStream_t s);

// Recombination as a dense contraction A (row fragments) x B^T (column
// fragments) over the 4^k cut terms, split along K.
struct GemmSide {
  uint32_t n;
  uint32_t frag[kMaxFrags];
  uint32_t shift[kMaxFrags];  // position of the fragment's row bits in the side's index
  uint32_t bits[kMaxFrags];
};
struct GemmArgs {
  uint32_t k, M, N;
  uint64_t K;
  // K index -> cut term: terms[kk] if set (sampled terms), else kk; each
  // term's row-side value is multiplied by tscale[kk] when set
  const uint64_t *terms;
  const double *tscale;
  uint32_t square;  // 1: every operand value squared (second moment of the sampled estimate)
  uint32_t lo_parts;  // fp32 mode: 1 = operands split hi + lo, three MFMA products; 0 = one fp32 product
  GemmSide L, R;
  uint32_t ident[kMaxFrags];  // 1 if the fragment's axes are cuts 0..k-1 in order (p_f(P) = P)
  RecombFrag f[kMaxFrags];
};
uint32_t gemm_splits(const GemmArgs &h);
// fp64 contractions with at most 32 rows take the skinny kernel (one
// column per thread, products summed in ascending term order) instead of
// 64 x 64 MFMA tiles; tiles, splits and the K range per split of either
bool contraction_skinny(const GemmArgs &h, bool fp32);
uint32_t skinny_cols(const GemmArgs &h);  // skinny kernel columns per thread (1, 2 or 4)
uint32_t gemm_tiles(const GemmArgs &h, bool skinny);
uint32_t contraction_splits(const GemmArgs &h, bool skinny);
uint64_t gemm_k_per_split(const GemmArgs &h, uint32_t splits, bool skinny);
// Batched contractions (one precision per launch): job j's workgroups
// [wg0, next wg0) are tiles x splits of its product, its reduction
// workgroups (256 outputs each) [rwg0, next rwg0).
struct GemmJob {
  const GemmArgs *args;
  double *partial;
  double *const *out;  // slot holding the output address (read when the job runs)
  uint64_t wg0, rwg0, k_per_split;
  uint32_t tiles, splits;
};
// skinny_rows: 0 for the MFMA tiles, else the row count M (1, 2, 4, ..., 32)
// and skinny_cpt the columns per thread (skinny_cols) every job of the list shares
// mode: 0 fp64, 1 fp32, 2 fp32 hi/lo (the MFMA tiles)
// gen: some contraction of the list has a side that is not one fragment
// read directly (gemm_general)
// (gen: lds = the largest gemm_fac_lds of the list)
hipError_t launch_gemm_batch(const GemmJob *d_jobs, uint32_t n_jobs, uint64_t total_wg, uint64_t total_rwg, int mode,
                             bool gen, size_t lds, uint32_t skinny_rows, uint32_t skinny_cpt, hipStream_t s);
bool gemm_general(const GemmArgs &h);
// Bytes of LDS the general tiles of contraction h take for operand factor
// tables.
size_t gemm_fac_lds(const GemmArgs &h);

hipError_t launch_recombine_gemm(const GemmArgs &h, const GemmArgs *d_args, bool fp32, double *partial,
                                 uint32_t splits, double *out, hipStream_t s,
                                 bool skinny = false);


// ------------------------------------------------- learned term proposal
enum MlpEpilogue : int { MLP_EPI_F32 = 0, MLP_EPI_BIAS_RELU = 1, MLP_EPI_MASK = 2 };
struct MlpGemm {
  const uint16_t *A;  // bf16, A(m, k) = A[m sam + k sak]
  uint64_t sam, sak;
  const uint16_t *B;  // bf16, B(k, n) = B[k sbk + n sbn]
  uint64_t sbk, sbn;
  uint64_t M;
  uint32_t N, K;
  void *C;             // fp32 (MLP_EPI_F32) or bf16
  uint64_t ldc;
  const float *bias;   // MLP_EPI_BIAS_RELU
  const uint16_t *mask;  // MLP_EPI_MASK: bf16 layer output, row stride ldm
  uint64_t ldm;
};
hipError_t launch_mlp_gemm(const MlpGemm &g, int epi, hipStream_t s);
hipError_t launch_head_forward(const uint16_t *H, uint32_t width, uint64_t rows, const uint16_t *w, const float *b,
                               float scale, float *y, hipStream_t s);
hipError_t launch_head_backward(const uint16_t *H, uint32_t width, uint64_t rows, const uint16_t *w, const float *y,
                                const float *t, float *dy, float *sq, uint16_t *dZ, hipStream_t s);
uint32_t colsum_chunks(uint64_t rows);
hipError_t launch_colsum(const uint16_t *X, uint32_t width, uint64_t rows, const float *sc, float *part, float *out,
                         hipStream_t s);
hipError_t launch_vsum(const float *x, uint64_t n, float *out, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, uint64_t n, float lr, float b1,
                       float b2, float c1, float c2, float eps, hipStream_t s);
hipError_t launch_to_bf16(const float *p, uint16_t *pb, uint64_t n, hipStream_t s);
hipError_t launch_gather_rows(const uint16_t *X, const float *y, uint64_t n, uint32_t width, uint32_t batch,
                              uint32_t step, uint64_t seed, int in_order, uint16_t *Xb, float *yb, hipStream_t s);

// The network regresses ln-weights divided by this scale (targets in
// [-1.04, 0]); its logits are the scale times its output.
constexpr float kLabelScale = 40.f;
// Per-circuit term model: fragment column norms and per-cut phi tables.
struct LearnedDev {
  uint32_t k, n_frags;
  const double *norm[kMaxFrags];  // n_f[p_f]
  uint32_t n_axes[kMaxFrags];
  uint32_t axis_cut[kMaxFrags][kMaxAxes];
  const double *phi;              // [cut][side: 0 up, 1 down][digit]
};
hipError_t launch_colnorm(const double *T, uint32_t rows, uint64_t ncols, double *out, hipStream_t s);
uint32_t share_chunks(uint32_t n_axes);
hipError_t launch_shares(const double *norm, uint32_t n_axes, double *part, double *shares, hipStream_t s);
hipError_t launch_phi(const double *shares, const int64_t *src, uint32_t k, double *phi, hipStream_t s);
hipError_t launch_features(const LearnedDev *L, const uint64_t *terms, uint64_t first, uint64_t n, uint32_t width,
                           uint16_t *X, hipStream_t s);
// The whole forward pass over term rows [first, first + n) in one launch:
// features from L, three ReLU layers (bf16 MFMA products, fp32
// accumulation in the same k order as mlp_gemm, bias, ReLU, bf16), the head
// y = scale (b4 + h3 . w4) summed as the separate head kernel does; the
// activations never leave the workgroup.  F = 64 inputs, H = 256.
struct MlpFused {
  const uint16_t *w1, *w2, *w3, *w4;  // bf16 [H][F], [H][H], [H][H], [H]
  const float *b1, *b2, *b3, *b4;
  uint32_t F, H;
};
hipError_t launch_mlp_logits_fused(const LearnedDev *L, const MlpFused &net, uint64_t first, uint64_t n, float scale,
                                   float *y, hipStream_t s);
hipError_t launch_labels(const LearnedDev *L, const uint64_t *terms, uint64_t first, uint64_t n, float *y, int kind,
                         hipStream_t s);
hipError_t launch_support(const LearnedDev *L, uint64_t K, uint64_t *flags, uint64_t *pos, uint64_t *scratch,
                          uint64_t cap, uint64_t *out, hipStream_t s);
uint64_t scan_scratch_words(uint64_t n);
hipError_t launch_scan_u64(uint64_t *x, uint64_t n, uint64_t *scratch, hipStream_t s);
uint32_t reduce_blocks(uint64_t n);
hipError_t launch_proposal(const float *logits, uint64_t n, double eps, float *mpart, double *spart, double *stats,
                           double *q, hipStream_t s);
// The error text of a call without a context (ccut_last_error(NULL)).
void set_call_error(const char *msg);
hipError_t launch_int_cdf(const double *q, uint64_t n, uint64_t *cdf, uint64_t *scratch, hipStream_t s);
hipError_t launch_sample_terms(const uint64_t *cdf, uint64_t K, uint64_t n, uint64_t seed, uint64_t cid,
                               uint64_t *out, hipStream_t s);
hipError_t launch_is_scale(const uint64_t *terms, const double *q, uint64_t n, double *scale, hipStream_t s);

}  // namespace ccut
