// Non-Clifford fragment variants on a dense fp64 state vector (the paper's
// exact backend for non-Clifford fragments, Sec. V-B).
//
// Variants of a fragment share everything but their preparations and their
// final basis rotations.  A workgroup simulates the fragment for one
// preparation combination (state in LDS, m <= 12 qubits: 64 KiB) and then
// rotates the state into one basis combination (small grids: one workgroup
// per preparation and basis combination) or, for large grids, into each
// basis combination in turn on a copy, and writes that variant's outcome
// distribution over the measured set.  Runs of one-qubit gates
// arrive fused into single 2x2 unitaries (G_U2).  Each distribution entry is
// reduced in a fixed order (deterministic).
#include "common.hpp"

namespace ccut {

namespace {


struct C2 {
  double re, im;
};

__device__ inline C2 cmul(C2 a, C2 b) { return C2{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline C2 cadd(C2 a, C2 b) { return C2{a.re + b.re, a.im + b.im}; }

// insert a zero bit at position t
__device__ inline uint32_t ins0(uint32_t k, uint32_t t) { return ((k >> t) << (t + 1)) | (k & ((1u << t) - 1)); }

__device__ void apply_gate(C2 *amp, uint32_t m, uint32_t kind, uint32_t a, uint32_t b, const double *mat) {
  const uint32_t N = 1u << m;
  const uint32_t half = N >> 1;
  const uint32_t ma = 1u << a;
  switch (kind) {
    case G_U2: {
      const C2 m00{mat[0], mat[1]}, m01{mat[2], mat[3]}, m10{mat[4], mat[5]}, m11{mat[6], mat[7]};
      for (uint32_t k = threadIdx.x; k < half; k += blockDim.x) {
        const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
        const C2 x = amp[i0], y = amp[i1];
        amp[i0] = cadd(cmul(m00, x), cmul(m01, y));
        amp[i1] = cadd(cmul(m10, x), cmul(m11, y));
      }
      break;
    }
    case G_H: {
      const double r = 0.70710678118654752440;
      for (uint32_t k = threadIdx.x; k < half; k += blockDim.x) {
        const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
        const C2 x = amp[i0], y = amp[i1];
        amp[i0] = C2{r * (x.re + y.re), r * (x.im + y.im)};
        amp[i1] = C2{r * (x.re - y.re), r * (x.im - y.im)};
      }
      break;
    }
    case G_X:
      for (uint32_t k = threadIdx.x; k < half; k += blockDim.x) {
        const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
        const C2 x = amp[i0];
        amp[i0] = amp[i1];
        amp[i1] = x;
      }
      break;
    case G_S: case G_SDG: {
      const double s = kind == G_S ? 1.0 : -1.0;
      for (uint32_t k = threadIdx.x; k < half; k += blockDim.x) {
        const uint32_t i1 = ins0(k, a) | ma;
        const C2 x = amp[i1];
        amp[i1] = C2{-s * x.im, s * x.re};
      }
      break;
    }
    case G_CX: {
      const uint32_t mb = 1u << b;
      for (uint32_t k = threadIdx.x; k < half; k += blockDim.x) {
        const uint32_t i0 = ins0(k, b);
        if (!(i0 & ma)) continue;
        const uint32_t i1 = i0 | mb;
        const C2 x = amp[i0];
        amp[i0] = amp[i1];
        amp[i1] = x;
      }
      break;
    }
    case G_CZ: {
      const uint32_t mb = 1u << b;
      for (uint32_t i = threadIdx.x; i < N; i += blockDim.x)
        if ((i & ma) && (i & mb)) amp[i] = C2{-amp[i].re, -amp[i].im};
      break;
    }
    default:
      break;
  }
  __syncthreads();
}

// The fused op stream (U2, CX, CZ and no-ops) on the state in LDS.  Each
// thread owns PPT amplitude pairs of every op and issues all their loads
// (and the op's 2x2 matrix, staged in LDS once per chunk of 16 ops) before
// any arithmetic; one barrier per op.
template <int PPT, int BS>
__device__ void sv_run_ops(C2 *amp, uint32_t m, const FragDev &F, C2 *s_mats) {
  const uint32_t half = (1u << m) >> 1;
  const uint32_t tid = threadIdx.x;
  const uint32_t n16 = (F.n_ops + 15) / 16;
  for (uint32_t g16 = 0; g16 < n16; ++g16) {
    // (the previous op's barrier has retired every read of the last chunk)
    if (tid < 64) s_mats[tid] = C2{F.mats[(size_t)g16 * 128 + 2 * tid], F.mats[(size_t)g16 * 128 + 2 * tid + 1]};
    __syncthreads();
    // one rolled op loop keeps the code small; the op word is a scalar load
    // issued when no LDS access is outstanding
#pragma unroll 1
    for (int t = 0; t < 16; ++t) {
      const uint32_t w = ((const g_u32 *)F.ops)[g16 * 16 + t];
      const uint32_t kind = op_kind(w);
      if (kind == G_NOP) continue;
      const uint32_t a = op_q0(w), b = op_q1(w);
      const uint32_t ma = 1u << a;
      if (kind == G_U2) {
        const C2 *M = s_mats + 4 * t;
        const C2 m00 = M[0], m01 = M[1], m10 = M[2], m11 = M[3];
        uint32_t i0[PPT];
        double xr[PPT], xi[PPT], yr[PPT], yi[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const uint32_t k = tid + p * BS;
          i0[p] = ins0(k < half ? k : 0, a);
          const C2 u = amp[i0[p]], v = amp[i0[p] | ma];
          xr[p] = u.re;
          xi[p] = u.im;
          yr[p] = v.re;
          yi[p] = v.im;
        }
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          if (tid + p * BS < half) {
            const C2 x{xr[p], xi[p]}, y{yr[p], yi[p]};
            amp[i0[p]] = cadd(cmul(m00, x), cmul(m01, y));
            amp[i0[p] | ma] = cadd(cmul(m10, x), cmul(m11, y));
          }
        }
      } else if (kind == G_CX) {
        // swap the target pair where the control bit is set
        const uint32_t mb = 1u << b;
        uint32_t i0[PPT];
        double xr[PPT], xi[PPT], yr[PPT], yi[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const uint32_t k = tid + p * BS;
          i0[p] = ins0(k < half ? k : 0, b);
          const C2 u = amp[i0[p]], v = amp[i0[p] | mb];
          xr[p] = u.re;
          xi[p] = u.im;
          yr[p] = v.re;
          yi[p] = v.im;
        }
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          if (tid + p * BS < half && (i0[p] & ma)) {
            amp[i0[p]] = C2{yr[p], yi[p]};
            amp[i0[p] | mb] = C2{xr[p], xi[p]};
          }
        }
      } else if (kind == G_CZ) {
        const uint32_t mb = 1u << b;
        for (uint32_t i = tid; i < 2 * half; i += BS)
          if ((i & ma) && (i & mb)) amp[i] = C2{-amp[i].re, -amp[i].im};
      }
      __syncthreads();
    }
  }
}

// split_bc: workgroup x runs preparation combination x / 3^n_out and only
// basis combination x mod 3^n_out (rotating its own state in place), so the
// basis combinations run side by side; otherwise workgroup x runs
// preparation combination x and every basis combination on a copy.
template <int PPT, int BS>
__global__ __launch_bounds__(BS) void sv_kernel(const FragDev F, double *__restrict__ dist, uint32_t split_bc) {
  extern __shared__ C2 smem_amp[];
  __shared__ C2 s_mats[64];
  const uint32_t m = F.m;
  const uint32_t N = 1u << m;
  const uint32_t tid = threadIdx.x;
  C2 *base = smem_amp;
  // preparation combination of this workgroup: digits of the input axes
  uint32_t n_out = 0;
  for (uint32_t j = 0; j < F.n_axes; ++j) n_out += F.axis_side[j] == 0;
  uint32_t n_bc = 1;
  for (uint32_t j = 0; j < n_out; ++j) n_bc *= 3;
  const uint32_t prep = split_bc ? blockIdx.x / n_bc : blockIdx.x;
  const uint32_t bc0 = split_bc ? blockIdx.x % n_bc : 0, bc1 = split_bc ? bc0 + 1 : n_bc;
  const bool copy = n_out && !split_bc;
  C2 *work = copy ? smem_amp + N : smem_amp;
  for (uint32_t i = tid; i < N; i += BS) base[i] = C2{i == 0 ? 1.0 : 0.0, 0.0};
  __syncthreads();
  uint64_t vin = 0;  // variant index contribution of the input digits
  {
    uint64_t pc = prep, stride = 1;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      if (F.axis_side[j] == 1) {
        const uint32_t d = (uint32_t)(pc & 3u);
        pc >>= 2;
        vin += d * stride;
        const uint32_t q = F.axis_local[j];
        if (d == 1) {
          apply_gate(base, m, G_X, q, 0, nullptr);
        } else if (d >= 2) {  // |+> = H|0>, |+i> = S H|0>
          apply_gate(base, m, G_H, q, 0, nullptr);
          if (d == 3) apply_gate(base, m, G_S, q, 0, nullptr);
        }
      }
      stride *= F.axis_radix[j];
    }
  }
  sv_run_ops<PPT, BS>(base, m, F, s_mats);
  // outcome distribution of every basis combination
  const uint32_t nm = F.n_meas;
  uint32_t mmask = 0;
  for (uint32_t j = 0; j < nm; ++j) mmask |= 1u << F.meas[j];
  const uint32_t outs = 1u << nm;
  for (uint32_t bc = bc0; bc < bc1; ++bc) {
    if (copy) {
      for (uint32_t i = tid; i < N; i += BS) work[i] = base[i];
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
          if (d == 1) apply_gate(work, m, G_SDG, q, 0, nullptr);
          if (d <= 1) apply_gate(work, m, G_H, q, 0, nullptr);
        }
        stride *= F.axis_radix[j];
      }
    }
    double *out = dist + v * outs;
    // outcome probabilities: |amp|^2 in place (reusing the work buffer as
    // N doubles), then a pairwise sum over each unmeasured qubit in turn
    // (fixed order, one barrier per qubit); the entry of outcome o is left
    // at the index with o's bits on the measured qubits and zeros elsewhere
    double pr[((1 << kMaxNcQubits) / BS)];
#pragma unroll
    for (int j = 0; j < ((1 << kMaxNcQubits) / BS); ++j) {
      const uint32_t i = tid + j * BS;
      pr[j] = 0.0;
      if (i < N) pr[j] = work[i].re * work[i].re + work[i].im * work[i].im;
    }
    __syncthreads();
    double *P = reinterpret_cast<double *>(work);
#pragma unroll
    for (int j = 0; j < ((1 << kMaxNcQubits) / BS); ++j) {
      const uint32_t i = tid + j * BS;
      if (i < N) P[i] = pr[j];
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

}  // namespace

hipError_t launch_sv(const FragDev &h, double *dist, hipStream_t s) {
  if (h.m > (uint32_t)kMaxNcQubits || h.n_meas > h.m) return hipErrorInvalidValue;
  uint32_t n_in = 0, n_out = 0;
  for (uint32_t j = 0; j < h.n_axes; ++j) (h.axis_side[j] ? n_in : n_out) += 1;
  // basis combinations get workgroups of their own while the grid stays
  // within about two workgroups per compute unit (each one repeats the
  // gate sequence, which costs nothing while the chip would idle)
  uint64_t n_bc = 1;
  for (uint32_t j = 0; j < n_out; ++j) n_bc *= 3;
  const uint64_t n_prep = 1ull << (2 * n_in);
  const bool split = n_out && n_prep * n_bc <= 512;
  const size_t lds = (size_t(1) << h.m) * sizeof(C2) * (n_out && !split ? 2 : 1);
  // one workgroup per preparation combination, sized to the state: 256
  // threads up to 9 qubits, then 512, then 1024 (several waves per SIMD
  // hide the LDS and fp64 latency); PPT amplitude pairs per thread per op
  auto kern = h.m <= 9 ? sv_kernel<1, 256> : h.m == 10 ? sv_kernel<1, 512> : h.m == 11 ? sv_kernel<1, 1024>
                                                                                   : sv_kernel<2, 1024>;
  const int bs = h.m <= 9 ? 256 : h.m == 10 ? 512 : 1024;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)(split ? n_prep * n_bc : n_prep)), dim3(bs), lds, s, h, dist,
                     (uint32_t)split);
  return hipGetLastError();
}

}  // namespace ccut
