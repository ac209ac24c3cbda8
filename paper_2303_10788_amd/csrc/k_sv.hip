// Non-Clifford fragment variants on a dense fp64 state vector (the paper's
// exact backend for non-Clifford fragments, Sec. V-B).
//
// Variants of a fragment share everything but their preparations and their
// final basis rotations.  A workgroup simulates the fragment for one
// preparation combination and then rotates the state into one basis
// combination (small grids: one workgroup per preparation and basis
// combination) or, for large grids, into each basis combination in turn on
// a copy, and writes that variant's outcome distribution over the measured
// set.
//
// The fragment is linear in its input state, and |+> = (|0> + |1>)/sqrt2,
// |+i> = (|0> + i|1>)/sqrt2.  So a fragment with quantum inputs is run only
// on the 2^n_in computational-basis inputs (evolve pass, final states to
// HBM), and the state of each of the 4^n_in preparation combinations is
// their linear combination (combine pass, which then rotates and sums the
// outcomes as above): 2^n_in instead of 4^n_in runs of the gate program.
//
// The state lives in registers while the gates run: amplitude index bits
// [0, RB) pick one of a thread's 2^RB registers, the next (up to) 6 bits the
// lane, the top bits the wave (sv_shape).  The host lays the gate stream out
// as a program over these bit positions (runs of one-qubit gates fused into
// one 2x2 unitary): a gate along a register bit is arithmetic on the
// thread's own registers, one along a lane bit exchanges amplitudes with the
// partner lane, diagonal gates, CZ and CX controls need no data movement,
// and a qubit needed on a wave bit is first swapped in through LDS (the only
// workgroup barrier besides program staging).  At the end the state goes to
// LDS in logical order for the basis rotations and the outcome sums.  Each
// distribution entry is reduced in a fixed order (deterministic).
#include "common.hpp"

// No implicit contraction: every fused multiply-add is written out, so the
// single-fragment and the batched kernel (the same body inlined in
// different code) round identically.
#pragma clang fp contract(off)

namespace ccut {

namespace {

struct C2 {
  double re, im;
};

__device__ inline C2 cmul(C2 a, C2 b) {
  return C2{__builtin_fma(a.re, b.re, -(a.im * b.im)), __builtin_fma(a.re, b.im, a.im * b.re)};
}
__device__ inline C2 cadd(C2 a, C2 b) { return C2{a.re + b.re, a.im + b.im}; }

// insert a zero bit at position t
__device__ inline uint32_t ins0(uint32_t k, uint32_t t) { return ((k >> t) << (t + 1)) | (k & ((1u << t) - 1)); }

// Basis rotations on the state in LDS (H, S^dagger), one barrier each.
__device__ void lds_h(C2 *amp, uint32_t m, uint32_t a) {
  const uint32_t half = (1u << m) >> 1, ma = 1u << a;
  const double r = 0.70710678118654752440;
  for (uint32_t k = threadIdx.x; k < half; k += blockDim.x) {
    const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
    const C2 x = amp[i0], y = amp[i1];
    amp[i0] = C2{r * (x.re + y.re), r * (x.im + y.im)};
    amp[i1] = C2{r * (x.re - y.re), r * (x.im - y.im)};
  }
  __syncthreads();
}

__device__ void lds_sdg(C2 *amp, uint32_t m, uint32_t a) {
  const uint32_t half = (1u << m) >> 1, ma = 1u << a;
  for (uint32_t k = threadIdx.x; k < half; k += blockDim.x) {
    const uint32_t i1 = ins0(k, a) | ma;
    const C2 x = amp[i1];
    amp[i1] = C2{x.im, -x.re};
  }
  __syncthreads();
}

constexpr uint32_t kStage = 64;  // program words staged in LDS at a time

// Partner-lane exchange of a thread's R amplitudes for a lane-bit op:
// lane ^ 1 and lane ^ 2 through DPP quad permutes (no LDS round trip),
// other masks through ds_bpermute with the byte address (lane ^ mask) * 4.
// All 4R moves of one op are issued back to back.
template <int MODE>
__device__ inline int xlane32(int v, int addr) {
  if constexpr (MODE == 0) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  else if constexpr (MODE == 1) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  else return __builtin_amdgcn_ds_bpermute(addr, v);
}

template <int R, int MODE>
__device__ inline void xlane_all(const double *re, const double *im, double *yr, double *yi, int addr) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t a = __builtin_bit_cast(uint64_t, re[r]), b = __builtin_bit_cast(uint64_t, im[r]);
    const uint32_t a0 = (uint32_t)xlane32<MODE>((int)(uint32_t)a, addr);
    const uint32_t a1 = (uint32_t)xlane32<MODE>((int)(uint32_t)(a >> 32), addr);
    const uint32_t b0 = (uint32_t)xlane32<MODE>((int)(uint32_t)b, addr);
    const uint32_t b1 = (uint32_t)xlane32<MODE>((int)(uint32_t)(b >> 32), addr);
    yr[r] = __builtin_bit_cast(double, ((uint64_t)a1 << 32) | a0);
    yi[r] = __builtin_bit_cast(double, ((uint64_t)b1 << 32) | b0);
  }
}

template <int R>
__device__ inline void xlane(const double *re, const double *im, double *yr, double *yi, uint32_t mask, int addr) {
  if (mask == 1)
    xlane_all<R, 0>(re, im, yr, yi, addr);
  else if (mask == 2)
    xlane_all<R, 1>(re, im, yr, yi, addr);
  else
    xlane_all<R, 2>(re, im, yr, yi, addr);
}

// c ? y : x on the bit patterns (exact, no branch)
__device__ inline double pick(bool c, double y, double x) {
  const uint64_t k = 0ull - (uint64_t)c;
  return __builtin_bit_cast(double, (__builtin_bit_cast(uint64_t, y) & k) | (__builtin_bit_cast(uint64_t, x) & ~k));
}

// A 2x2 unitary along register bit P: pairs (r, r | 2^P) of this thread.
template <int RB, int P>
__device__ inline void u2_reg_at(double *re, double *im, C2 m00, C2 m01, C2 m10, C2 m11) {
  if constexpr (P < RB) {
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
      if (r & (1 << P)) continue;
      const int s = r | (1 << P);
      const C2 x{re[r], im[r]}, y{re[s], im[s]};
      const C2 u = cadd(cmul(m00, x), cmul(m01, y)), v = cadd(cmul(m10, x), cmul(m11, y));
      re[r] = u.re;
      im[r] = u.im;
      re[s] = v.re;
      im[s] = v.im;
    }
  }
}

template <int RB>
__device__ inline void u2_reg(double *re, double *im, uint32_t p, C2 m00, C2 m01, C2 m10, C2 m11) {
  switch (p) {
    case 0: u2_reg_at<RB, 0>(re, im, m00, m01, m10, m11); break;
    case 1: u2_reg_at<RB, 1>(re, im, m00, m01, m10, m11); break;
    default: break;
  }
}

// CX with its target on register bit P; `base` is the index of register 0.
template <int RB, int P>
__device__ inline void cx_reg_at(double *re, double *im, uint32_t base, uint32_t ctrl) {
  if constexpr (P < RB) {
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
      if (r & (1 << P)) continue;
      const int s = r | (1 << P);
      const bool c = ((base | (uint32_t)r) >> ctrl) & 1u;
      const double xr = re[r], xi = im[r], yr = re[s], yi = im[s];
      re[r] = pick(c, yr, xr);
      im[r] = pick(c, yi, xi);
      re[s] = pick(c, xr, yr);
      im[s] = pick(c, xi, yi);
    }
  }
}

template <int RB>
__device__ inline void cx_reg(double *re, double *im, uint32_t base, uint32_t ctrl, uint32_t p) {
  switch (p) {
    case 0: cx_reg_at<RB, 0>(re, im, base, ctrl); break;
    case 1: cx_reg_at<RB, 1>(re, im, base, ctrl); break;
    default: break;
  }
}

// split_bc: workgroup x runs preparation combination x / 3^n_out and only
// basis combination x mod 3^n_out (rotating its own state in place);
// otherwise workgroup x runs preparation combination x and every basis
// combination on a copy.  blockDim.x = 64 * 2^wb (sv_shape, up to 1024),
// RB register bits per thread.
template <class T>
__device__ inline const T *uniform_ptr(const T *p) {
  const uint64_t u = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (const T *)(((uint64_t)hi << 32) | lo);
}

// One state buffer in LDS instead of two: when no basis-combination copy
// needs the second one and the state is large enough that halving the LDS
// lets more workgroups share a compute unit.  Swaps then take a second
// barrier (their writes must wait for the previous swap's reads).
__host__ __device__ inline bool sv_single_buffer(uint32_t m, bool copy) { return !copy && m >= 11; }

// Passes of sv_body: the whole variant (fragments without quantum inputs),
// the evolve pass (computational-basis inputs, final state to `states`) and
// the combine pass (no gate program: a preparation combination's state from
// `states`, then the basis rotations and outcome sums).
enum : uint32_t { SV_FULL = 0, SV_EVOLVE = 1, SV_COMBINE = 2 };

// The basis rotations and outcome distributions of one preparation
// combination whose state is in S (logical order); vin = the variant-index
// contribution of its input digits.
__device__ void sv_outcomes(const FragDev &F, C2 *S, C2 *work, bool copy, uint32_t bc0, uint32_t bc1, uint64_t vin,
                            double *__restrict__ dist, uint32_t R);

template <int RB>
__device__ __attribute__((always_inline)) void sv_body(const FragDev &F, double *__restrict__ dist, uint32_t split_bc,
                                                       uint32_t blk, C2 *smem, uint32_t mode, C2 *__restrict__ states) {
  constexpr int R = 1 << RB;
  // the descriptor's scalars in scalar registers (uniform across the
  // workgroup; read from memory they would hold vector registers)
  const uint32_t m = __builtin_amdgcn_readfirstlane(F.m);
  const uint32_t n_ops = __builtin_amdgcn_readfirstlane(F.n_ops);
  const uint32_t *ops = uniform_ptr(F.ops);
  const double *mats = uniform_ptr(F.mats);
  const uint32_t N = 1u << m;
  const uint32_t BS = blockDim.x;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t base = (wave << (RB + 6)) | (lane << RB);  // index of register 0
  const bool live = base < N;  // fewer than 64 amplitudes: the upper lanes idle
  uint32_t n_out = 0;
  for (uint32_t j = 0; j < F.n_axes; ++j) n_out += F.axis_side[j] == 0;
  const bool copy = mode != SV_EVOLVE && n_out && !split_bc;
  const bool single = sv_single_buffer(m, copy);
  C2 *buf0 = smem, *buf1 = single ? smem : smem + N;
  double *s_mats = reinterpret_cast<double *>(smem + (single ? 1 : 2) * N);
  uint32_t n_bc = 1;
  for (uint32_t j = 0; j < n_out; ++j) n_bc *= 3;
  const uint32_t prep = split_bc ? blk / n_bc : blk;
  const uint32_t bc0 = split_bc ? blk % n_bc : 0, bc1 = split_bc ? bc0 + 1 : n_bc;

  if (mode == SV_COMBINE) {
    // the preparation combination's state from the basis-input states:
    // psi_s = h^(#superposed inputs) sum_b phase(s, b) psi_b over the inputs b
    // compatible with s (digit 0 or 1: that bit; + or +i: both, the second
    // times 1 or i), summed in ascending b
    uint32_t n_in = 0, fixed = 0, sup = 0, imul = 0;
    uint64_t vin = 0, stride = 1;
    {
      uint64_t pc = prep;
      for (uint32_t j = 0; j < F.n_axes; ++j) {
        if (F.axis_side[j] == 1) {
          const uint32_t d = (uint32_t)(pc & 3u);
          pc >>= 2;
          vin += d * stride;
          if (d == 1) fixed |= 1u << n_in;
          if (d >= 2) sup |= 1u << n_in;
          if (d == 3) imul |= 1u << n_in;
          ++n_in;
        }
        stride *= F.axis_radix[j];
      }
    }
    double scale = 1.0;
    for (uint32_t j = 0; j < n_in; ++j)
      if ((sup >> j) & 1u) scale *= 0.70710678118654752440;
    for (uint32_t i = tid; i < N; i += BS) {
      double ar = 0.0, ai = 0.0;
      // enumerate the subsets of `sup` in ascending order of b = fixed | sub
      uint32_t sub = 0;
      do {
        const uint32_t b = fixed | sub;
        const __attribute__((address_space(1))) double *sp =
            (const __attribute__((address_space(1))) double *)states + 2 * ((size_t)b * N + i);
        const C2 v{sp[0], sp[1]};
        // the number of +i digits whose input bit is 1 sets the phase i^k
        const uint32_t k = __popc(sub & imul) & 3u;
        const double vr = k == 0 ? v.re : k == 1 ? -v.im : k == 2 ? -v.re : v.im;
        const double vi = k == 0 ? v.im : k == 1 ? v.re : k == 2 ? -v.im : -v.re;
        ar += vr;
        ai += vi;
        sub = (sub - sup) & sup;
      } while (sub);
      buf0[i] = C2{ar * scale, ai * scale};
    }
    __syncthreads();
    sv_outcomes(F, buf0, copy ? buf1 : buf0, copy, bc0, bc1, vin, dist, R);
    return;
  }

  // prepared product state: |0>, |1>, |+> = H|0> or |+i> = S H|0> on each
  // quantum input (digit of this preparation combination; in the evolve
  // pass bit j of the workgroup index is input j's computational-basis
  // value), |0> elsewhere
  double re[R], im[R];
  uint64_t vin = 0;  // variant index contribution of the input digits
  {
    uint32_t imask = 0;
    for (uint32_t j = 0; j < F.n_axes; ++j)
      if (F.axis_side[j] == 1) imask |= 1u << F.axis_local[j];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      re[r] = live && !((base | (uint32_t)r) & ~imask) ? 1.0 : 0.0;
      im[r] = 0.0;
    }
    const double h = 0.70710678118654752440;
    uint64_t pc = prep, stride = 1;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      if (F.axis_side[j] == 1) {
        const uint32_t d = mode == SV_EVOLVE ? (uint32_t)(pc & 1u) : (uint32_t)(pc & 3u);
        pc >>= mode == SV_EVOLVE ? 1 : 2;
        vin += d * stride;
        const uint32_t q = F.axis_local[j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const bool b = ((base | (uint32_t)r) >> q) & 1u;
          if (d == 0 && b) re[r] = im[r] = 0.0;
          if (d == 1 && !b) re[r] = im[r] = 0.0;
          if (d >= 2) {
            const double xr = re[r] * h, xi = im[r] * h;
            const bool rot = d == 3 && b;  // times i
            re[r] = rot ? -xi : xr;
            im[r] = rot ? xr : xi;
          }
        }
      }
      stride *= F.axis_radix[j];
    }
  }

  // the program
  uint64_t layout = 0;
  for (uint32_t q = 0; q < m; ++q) layout |= (uint64_t)q << (4 * q);
  uint32_t cur = 0;  // swap buffer of the next SV_SWAP
  for (uint32_t c0 = 0; c0 < n_ops; c0 += kStage) {
    const uint32_t cn = min(kStage, n_ops - c0);
    // lane t of every wave holds op word t of the chunk (read with
    // readlane: no LDS round trip per op); the matrices are staged in LDS
    // with every load of a thread issued before its first store
    const uint32_t myw = lane < cn ? ops[c0 + lane] : 0u;
    double mt[8 * kStage / 64];
#pragma unroll
    for (uint32_t k = 0; k < 8 * kStage / 64; ++k) {
      const uint32_t i = tid + k * BS;
      mt[k] = i < 8 * cn ? mats[(size_t)8 * c0 + i] : 0.0;
    }
    __syncthreads();  // every wave is done with the previous chunk
#pragma unroll
    for (uint32_t k = 0; k < 8 * kStage / 64; ++k) {
      const uint32_t i = tid + k * BS;
      if (i < 8 * cn) s_mats[i] = mt[k];
    }
    __syncthreads();
    // the matrix of op t + 1 (if it has one) is read while op t runs
    uint32_t wn = __builtin_amdgcn_readlane(myw, 0);
    double Mn[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) Mn[e] = 0.0;
    if (op_kind(wn) == SV_U2 || op_kind(wn) == SV_DIAG || op_kind(wn) == SV_END) {
#pragma unroll
      for (int e = 0; e < 8; ++e) Mn[e] = s_mats[e];
    }
#pragma unroll 1
    for (uint32_t t = 0; t < cn; ++t) {
      const uint32_t w = wn;
      double M[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) M[e] = Mn[e];
      if (t + 1 < cn) {
        wn = __builtin_amdgcn_readlane(myw, t + 1);
        const uint32_t kn = op_kind(wn);
        if (kn == SV_U2 || kn == SV_DIAG || kn == SV_END) {
#pragma unroll
          for (int e = 0; e < 8; ++e) Mn[e] = s_mats[8 * (t + 1) + e];
        }
      }
      const uint32_t kind = op_kind(w), a = op_q0(w), b = op_q1(w);
      switch (kind) {
        case SV_U2: {
          const C2 m00{M[0], M[1]}, m01{M[2], M[3]}, m10{M[4], M[5]}, m11{M[6], M[7]};
          if (a < (uint32_t)RB) {
            u2_reg<RB>(re, im, a, m00, m01, m10, m11);
          } else {
            const uint32_t mask = 1u << (a - RB);
            const int addr = (int)((lane ^ mask) << 2);
            const bool hi = lane & mask;
            const C2 k0 = hi ? m11 : m00, k1 = hi ? m10 : m01;  // own and partner coefficients
            double yr[R], yi[R];
            xlane<R>(re, im, yr, yi, mask, addr);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const C2 u = cadd(cmul(k0, C2{re[r], im[r]}), cmul(k1, C2{yr[r], yi[r]}));
              re[r] = u.re;
              im[r] = u.im;
            }
          }
          break;
        }
        case SV_DIAG: {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const bool c = ((base | (uint32_t)r) >> a) & 1u;
            const C2 d{pick(c, M[6], M[0]), pick(c, M[7], M[1])};
            const C2 u = cmul(d, C2{re[r], im[r]});
            re[r] = u.re;
            im[r] = u.im;
          }
          break;
        }
        case SV_CX: {
          if (b < (uint32_t)RB) {
            cx_reg<RB>(re, im, base, a, b);
          } else {
            const uint32_t mask = 1u << (b - RB);
            const int addr = (int)((lane ^ mask) << 2);
            double yr[R], yi[R];
            xlane<R>(re, im, yr, yi, mask, addr);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const bool c = ((base | (uint32_t)r) >> a) & 1u;
              re[r] = pick(c, yr[r], re[r]);
              im[r] = pick(c, yi[r], im[r]);
            }
          }
          break;
        }
        case SV_CZ: {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const uint32_t i = base | (uint32_t)r;
            const bool c = (i >> a) & (i >> b) & 1u;
            re[r] = pick(c, -re[r], re[r]);
            im[r] = pick(c, -im[r], im[r]);
          }
          break;
        }
        case SV_SWAP: {
          // amplitude i moves to i with bits a and b exchanged
          C2 *B = cur ? buf1 : buf0;
          if (single) __syncthreads();  // every read of the previous swap is done
          if (live) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const uint32_t i = base | (uint32_t)r;
              const uint32_t x = ((i >> a) ^ (i >> b)) & 1u;
              B[i ^ ((x << a) | (x << b))] = C2{re[r], im[r]};
            }
          }
          __syncthreads();
          if (live) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const C2 v = B[base | (uint32_t)r];
              re[r] = v.re;
              im[r] = v.im;
            }
          }
          cur ^= 1u;  // the next swap writes the other buffer, so no second barrier
          break;
        }
        case SV_END:
          layout = (uint64_t)__double_as_longlong(M[0]);
          break;
        default:
          break;
      }
    }
  }
  // the state in logical order: bit q of the logical index is the physical
  // bit at position layout[q]; the evolve pass writes it to HBM
  if (mode == SV_EVOLVE) {
    if (live) {
      C2 *dst = states + (size_t)blk * N;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = base | (uint32_t)r;
        uint32_t L = 0;
        for (uint32_t q = 0; q < m; ++q) L |= ((i >> ((layout >> (4 * q)) & 15u)) & 1u) << q;
        dst[L] = C2{re[r], im[r]};
      }
    }
    return;
  }
  C2 *S = cur ? buf1 : buf0;
  if (single) __syncthreads();  // the last swap's reads are done
  if (live) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = base | (uint32_t)r;
      uint32_t L = 0;
      for (uint32_t q = 0; q < m; ++q) L |= ((i >> ((layout >> (4 * q)) & 15u)) & 1u) << q;
      S[L] = C2{re[r], im[r]};
    }
  }
  __syncthreads();
  sv_outcomes(F, S, copy ? (cur ? buf0 : buf1) : S, copy, bc0, bc1, vin, dist, R);
}

__device__ void sv_outcomes(const FragDev &F, C2 *S, C2 *work, bool copy, uint32_t bc0, uint32_t bc1, uint64_t vin,
                            double *__restrict__ dist, uint32_t R) {
  const uint32_t m = F.m, N = 1u << m, BS = blockDim.x, tid = threadIdx.x;
  // outcome distribution of every basis combination
  const uint32_t nm = F.n_meas;
  uint32_t mmask = 0;
  for (uint32_t j = 0; j < nm; ++j) mmask |= 1u << F.meas[j];
  const uint32_t outs = 1u << nm;
  for (uint32_t bc = bc0; bc < bc1; ++bc) {
    if (copy) {
      for (uint32_t i = tid; i < N; i += BS) work[i] = S[i];
      __syncthreads();
    }
    uint64_t v = vin;
    {
      uint32_t t = bc;
      uint64_t stride = 1;
      for (uint32_t j = 0; j < F.n_axes; ++j) {
        if (F.axis_side[j] == 0) {
          const uint32_t d = t % 3;  // X: H; Y: S^dag then H; Z: nothing
          t /= 3;
          v += d * stride;
          const uint32_t q = F.axis_local[j];
          if (d == 1) lds_sdg(work, m, q);
          if (d <= 1) lds_h(work, m, q);
        }
        stride *= F.axis_radix[j];
      }
    }
    // stored through a global pointer (a generic store would hold up the
    // next LDS read until it completes)
    __attribute__((address_space(1))) double *out = (__attribute__((address_space(1))) double *)(dist + v * outs);
    // outcome probabilities: |amp|^2 in place (the work buffer as N
    // doubles; N = BS * R, so each thread holds at most R of them), then a
    // pairwise sum over each unmeasured qubit in turn (fixed order, one
    // barrier per qubit); the entry of outcome o is left at the index with
    // o's bits on the measured qubits and zeros elsewhere
    double pr[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t i = tid + j * BS;
      pr[j] = 0.0;
      if (j < R && i < N) pr[j] = work[i].re * work[i].re + work[i].im * work[i].im;
    }
    __syncthreads();
    double *P = reinterpret_cast<double *>(work);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t i = tid + j * BS;
      if (j < R && i < N) P[i] = pr[j];
    }
    __syncthreads();
    for (uint32_t q = 0; q < m; ++q) {
      if (mmask & (1u << q)) continue;
      const uint32_t mq = 1u << q;
      for (uint32_t k = tid; k < N / 2; k += BS) {
        const uint32_t i0 = ins0(k, q);
        P[i0] += P[i0 | mq];
      }
      __syncthreads();
    }
    for (uint32_t o = tid; o < outs; o += BS) {
      uint32_t idx = 0;
      for (uint32_t j = 0; j < nm; ++j) idx |= ((o >> j) & 1u) << F.meas[j];
      out[o] = P[idx];
    }
    __syncthreads();  // the next basis combination overwrites the work buffer
  }
}

template <int RB>
__global__ __launch_bounds__(1024) void sv_kernel(const FragDev F, double *__restrict__ dist, uint32_t split_bc,
                                                  uint32_t mode, C2 *__restrict__ states) {
  extern __shared__ C2 smem[];
  sv_body<RB>(F, dist, split_bc, blockIdx.x, smem, mode, states);
}

// Many fragments of one shape: workgroup x runs workgroup x - wg0 of the
// job holding x.
template <int RB>
__global__ __launch_bounds__(1024) void sv_batch_kernel(const FragDev *__restrict__ descs, const SvJob *__restrict__ jobs,
                                                        uint32_t n_jobs) {
  extern __shared__ C2 smem[];
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (jobs[mid].wg0 <= blockIdx.x) lo = mid;
    else hi = mid;
  }
  // the job's fields are workgroup-uniform: keep them in scalar registers
  const SvJob &J = jobs[__builtin_amdgcn_readfirstlane(lo)];
  const uint32_t desc = __builtin_amdgcn_readfirstlane(J.desc), split = __builtin_amdgcn_readfirstlane(J.split);
  const uint32_t mode = __builtin_amdgcn_readfirstlane(J.mode);
  const uint32_t blk = __builtin_amdgcn_readfirstlane((uint32_t)(blockIdx.x - J.wg0));
  double *dist = const_cast<double *>(uniform_ptr(J.dist));
  C2 *states = reinterpret_cast<C2 *>(const_cast<double *>(uniform_ptr(J.states)));
  sv_body<RB>(descs[desc], dist, split, blk, smem, mode, states);
}

}  // namespace

uint32_t sv_inputs(const FragDev &h) {
  uint32_t n_in = 0;
  for (uint32_t j = 0; j < h.n_axes; ++j) n_in += h.axis_side[j] == 1;
  return n_in;
}

// A fragment with cut axes runs in two passes: the gate program once per
// computational-basis input (the only run without inputs), then one
// workgroup per preparation and basis combination from the stored states
// (no workgroup repeats the program for a basis combination).  Fragments
// without axes run in one pass.
size_t sv_states_bytes(const FragDev &h) {
  return h.n_axes ? ((size_t)1 << (sv_inputs(h) + h.m)) * sizeof(C2) : 0;
}

void sv_pass_shape(const FragDev &h, uint32_t pass, uint64_t &n_wg, uint32_t &block, size_t &lds, bool &split) {
  if (pass == SV_EVOLVE) {
    // one workgroup per computational-basis input; the gate program needs
    // the swap buffers and the staged matrices, no basis-rotation copy
    n_wg = 1ull << sv_inputs(h);
    block = 64u << sv_shape(h.m).wb;
    split = false;
    lds = (size_t(sv_single_buffer(h.m, false) ? 1 : 2) << h.m) * sizeof(C2) + kStage * 8 * sizeof(double);
    return;
  }
  sv_launch_shape(h, n_wg, block, lds, split);
  if (pass == SV_COMBINE) {
    // no gate program: one workgroup per preparation and basis combination,
    // one state buffer each
    const uint32_t n_in = sv_inputs(h), n_out = h.n_axes - n_in;
    uint64_t n_bc = 1;
    for (uint32_t j = 0; j < n_out; ++j) n_bc *= 3;
    split = n_out != 0;
    n_wg = (1ull << (2 * n_in)) * n_bc;
    lds = ((size_t)1 << h.m) * sizeof(C2);
  }
}

void sv_launch_shape(const FragDev &h, uint64_t &n_wg, uint32_t &block, size_t &lds, bool &split) {
  uint32_t n_in = 0, n_out = 0;
  for (uint32_t j = 0; j < h.n_axes; ++j) (h.axis_side[j] ? n_in : n_out) += 1;
  // basis combinations get workgroups of their own while the grid stays
  // within about two workgroups per compute unit (each one repeats the
  // gate sequence, which costs nothing while the chip would idle)
  uint64_t n_bc = 1;
  for (uint32_t j = 0; j < n_out; ++j) n_bc *= 3;
  const uint64_t n_prep = 1ull << (2 * n_in);
  split = n_out && n_prep * n_bc <= 512;
  n_wg = split ? n_prep * n_bc : n_prep;
  block = 64u << sv_shape(h.m).wb;
  // two state buffers (swaps alternate between them; the copy mode uses the
  // second for the rotated copy), or one, and the staged matrices of a
  // program chunk
  const bool copy = n_out && !split;
  lds = (size_t(sv_single_buffer(h.m, copy) ? 1 : 2) << h.m) * sizeof(C2) + kStage * 8 * sizeof(double);
}

hipError_t launch_sv_batch(const FragDev *descs, const SvJob *jobs, uint32_t n_jobs, uint64_t total_wg, uint32_t m,
                           size_t lds, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  if (m == 0 || m > (uint32_t)kMaxNcQubits || total_wg > 0x7FFFFFFFull || lds > 160 * 1024)
    return hipErrorInvalidValue;
  const SvShape sh = sv_shape(m);
  const dim3 grid((unsigned)total_wg), block(64u << sh.wb);
  const void *kern = sh.rb == 0 ? (const void *)sv_batch_kernel<0>
                     : sh.rb == 1 ? (const void *)sv_batch_kernel<1>
                                  : (const void *)sv_batch_kernel<2>;
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  switch (sh.rb) {
    case 0: hipLaunchKernelGGL(sv_batch_kernel<0>, grid, block, lds, s, descs, jobs, n_jobs); break;
    case 1: hipLaunchKernelGGL(sv_batch_kernel<1>, grid, block, lds, s, descs, jobs, n_jobs); break;
    default: hipLaunchKernelGGL(sv_batch_kernel<2>, grid, block, lds, s, descs, jobs, n_jobs); break;
  }
  return hipGetLastError();
}

static hipError_t launch_sv_pass(const FragDev &h, double *dist, uint32_t pass, C2 *states, hipStream_t s) {
  uint64_t n_wg;
  uint32_t bs;
  size_t lds;
  bool split;
  sv_pass_shape(h, pass, n_wg, bs, lds, split);
  if (lds > 160 * 1024 || n_wg > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const SvShape sh = sv_shape(h.m);
  const void *kern = sh.rb == 0 ? (const void *)sv_kernel<0>
                     : sh.rb == 1 ? (const void *)sv_kernel<1>
                                  : (const void *)sv_kernel<2>;
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)n_wg), block(bs);
  switch (sh.rb) {
    case 0: hipLaunchKernelGGL(sv_kernel<0>, grid, block, lds, s, h, dist, (uint32_t)split, pass, states); break;
    case 1: hipLaunchKernelGGL(sv_kernel<1>, grid, block, lds, s, h, dist, (uint32_t)split, pass, states); break;
    default: hipLaunchKernelGGL(sv_kernel<2>, grid, block, lds, s, h, dist, (uint32_t)split, pass, states); break;
  }
  return hipGetLastError();
}

hipError_t launch_sv(const FragDev &h, double *dist, void *states, hipStream_t s) {
  if (h.m == 0 || h.m > (uint32_t)kMaxNcQubits || h.n_meas > h.m) return hipErrorInvalidValue;
  if (h.n_axes == 0) return launch_sv_pass(h, dist, SV_FULL, nullptr, s);
  if (!states) return hipErrorInvalidValue;
  hipError_t e = launch_sv_pass(h, dist, SV_EVOLVE, static_cast<C2 *>(states), s);
  if (e != hipSuccess) return e;
  return launch_sv_pass(h, dist, SV_COMBINE, static_cast<C2 *>(states), s);
}

}  // namespace ccut
