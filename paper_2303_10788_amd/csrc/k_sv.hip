// Non-Clifford fragment variants on a dense fp64 state vector (the paper's
// exact backend for non-Clifford fragments, Sec. V-B).
//
// Variants of a fragment share everything but their preparations and their
// final basis rotations, so one workgroup simulates the fragment once per
// preparation combination (state in LDS, m <= 12 qubits: 64 KiB) and then,
// for each basis combination, rotates a copy and writes that variant's
// outcome distribution over the measured set.  Runs of one-qubit gates
// arrive fused into single 2x2 unitaries (G_U2).  Each distribution entry is
// reduced in a fixed order (deterministic).
#include "common.hpp"

namespace ccut {

namespace {

constexpr int kSvBlock = 256;

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
      for (uint32_t k = threadIdx.x; k < half; k += kSvBlock) {
        const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
        const C2 x = amp[i0], y = amp[i1];
        amp[i0] = cadd(cmul(m00, x), cmul(m01, y));
        amp[i1] = cadd(cmul(m10, x), cmul(m11, y));
      }
      break;
    }
    case G_H: {
      const double r = 0.70710678118654752440;
      for (uint32_t k = threadIdx.x; k < half; k += kSvBlock) {
        const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
        const C2 x = amp[i0], y = amp[i1];
        amp[i0] = C2{r * (x.re + y.re), r * (x.im + y.im)};
        amp[i1] = C2{r * (x.re - y.re), r * (x.im - y.im)};
      }
      break;
    }
    case G_X:
      for (uint32_t k = threadIdx.x; k < half; k += kSvBlock) {
        const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
        const C2 x = amp[i0];
        amp[i0] = amp[i1];
        amp[i1] = x;
      }
      break;
    case G_S: case G_SDG: {
      const double s = kind == G_S ? 1.0 : -1.0;
      for (uint32_t k = threadIdx.x; k < half; k += kSvBlock) {
        const uint32_t i1 = ins0(k, a) | ma;
        const C2 x = amp[i1];
        amp[i1] = C2{-s * x.im, s * x.re};
      }
      break;
    }
    case G_CX: {
      const uint32_t mb = 1u << b;
      for (uint32_t k = threadIdx.x; k < half; k += kSvBlock) {
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
      for (uint32_t i = threadIdx.x; i < N; i += kSvBlock)
        if ((i & ma) && (i & mb)) amp[i] = C2{-amp[i].re, -amp[i].im};
      break;
    }
    default:
      break;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSvBlock) void sv_kernel(const FragDev F, double *__restrict__ dist) {
  extern __shared__ C2 smem_amp[];
  __shared__ double part[kSvBlock];
  __shared__ double s_mats[16 * 8];
  const uint32_t m = F.m;
  const uint32_t N = 1u << m;
  const uint32_t tid = threadIdx.x;
  C2 *base = smem_amp;
  // preparation combination of this workgroup: digits of the input axes
  uint32_t n_out = 0;
  for (uint32_t j = 0; j < F.n_axes; ++j) n_out += F.axis_side[j] == 0;
  C2 *work = n_out ? smem_amp + N : smem_amp;
  for (uint32_t i = tid; i < N; i += kSvBlock) base[i] = C2{i == 0 ? 1.0 : 0.0, 0.0};
  __syncthreads();
  uint64_t vin = 0;  // variant index contribution of the input digits
  {
    uint64_t pc = blockIdx.x, stride = 1;
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
  // the fused 2x2 matrices of a chunk of 16 ops are staged in LDS (one
  // coalesced load) so gates read them with broadcast LDS reads
  for (uint32_t g16 = 0; g16 < (F.n_ops + 15) / 16; ++g16) {
    for (uint32_t i = tid; i < 16 * 8; i += kSvBlock) s_mats[i] = F.mats[(size_t)g16 * 128 + i];
    __syncthreads();
    const Ops16 o = load_ops16(F.ops, g16);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const uint32_t w = o.w[t];
      if (op_kind(w) == G_NOP) continue;
      apply_gate(base, m, op_kind(w), op_q0(w), op_q1(w), s_mats + 8 * t);
    }
  }
  // outcome distribution of every basis combination
  const uint32_t nm = F.n_meas;
  uint32_t mmask = 0;
  for (uint32_t j = 0; j < nm; ++j) mmask |= 1u << F.meas[j];
  const uint32_t rest = m - nm;
  const uint32_t outs = 1u << nm;
  const uint32_t tpo = outs >= (uint32_t)kSvBlock ? 1u : (uint32_t)kSvBlock / outs;  // threads per output
  uint32_t n_bc = 1;
  for (uint32_t j = 0; j < n_out; ++j) n_bc *= 3;
  for (uint32_t bc = 0; bc < n_bc; ++bc) {
    if (n_out) {
      for (uint32_t i = tid; i < N; i += kSvBlock) work[i] = base[i];
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
    // entry o sums |amp|^2 over the unmeasured bits; tpo threads per entry
    // take interleaved parts, then one thread adds the parts in order
    for (uint32_t o0 = 0; o0 < outs; o0 += kSvBlock / tpo) {
      const uint32_t o = o0 + tid / tpo, part_id = tid % tpo;
      double acc = 0.0;
      if (o < outs) {
        uint32_t basei = 0;
        for (uint32_t j = 0; j < nm; ++j) basei |= ((o >> j) & 1u) << F.meas[j];
        for (uint32_t r = part_id; r < (1u << rest); r += tpo) {
          uint32_t idx = basei, rr = r;
          for (uint32_t q = 0; q < m; ++q) {
            if (mmask & (1u << q)) continue;
            idx |= (rr & 1u) << q;
            rr >>= 1;
          }
          const C2 a = work[idx];
          acc += a.re * a.re + a.im * a.im;
        }
      }
      part[tid] = acc;
      __syncthreads();
      if (part_id == 0 && o < outs) {
        double s = 0.0;
        for (uint32_t t = 0; t < tpo; ++t) s += part[tid + t];
        out[o] = s;
      }
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t launch_sv(const FragDev &h, double *dist, hipStream_t s) {
  if (h.m > (uint32_t)kMaxNcQubits || h.n_meas > h.m) return hipErrorInvalidValue;
  uint32_t n_in = 0, n_out = 0;
  for (uint32_t j = 0; j < h.n_axes; ++j) (h.axis_side[j] ? n_in : n_out) += 1;
  const size_t lds = (size_t(1) << h.m) * sizeof(C2) * (n_out ? 2 : 1);
  hipError_t e = hipFuncSetAttribute((const void *)sv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const uint64_t n_prep = 1ull << (2 * n_in);
  hipLaunchKernelGGL(sv_kernel, dim3((unsigned)n_prep), dim3(kSvBlock), lds, s, h, dist);
  return hipGetLastError();
}

}  // namespace ccut
