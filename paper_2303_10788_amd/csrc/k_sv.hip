// Non-Clifford fragment variants on a dense fp64 state vector (the paper's
// exact backend for non-Clifford fragments, Sec. V-B).  One workgroup per
// variant; the 2^m complex amplitudes (m <= 12: 64 KiB) stay in LDS for
// the whole circuit.  Output: the variant's outcome distribution over its
// measured set, each entry summed over the unmeasured bits in ascending
// order (deterministic).
#include "common.hpp"

namespace ccut {

namespace {

constexpr int kSvBlock = 256;

struct C2 {
  double re, im;
};

__device__ inline C2 cmul(C2 a, C2 b) { return C2{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// insert a zero bit at position t
__device__ inline uint32_t ins0(uint32_t k, uint32_t t) { return ((k >> t) << (t + 1)) | (k & ((1u << t) - 1)); }

__device__ void apply_gate(C2 *amp, uint32_t m, uint32_t kind, uint32_t a, uint32_t b, double theta) {
  const uint32_t N = 1u << m;
  const uint32_t half = N >> 1;
  const uint32_t ma = 1u << a;
  switch (kind) {
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
    case G_Y:  // Y = [[0, -i], [i, 0]]
      for (uint32_t k = threadIdx.x; k < half; k += kSvBlock) {
        const uint32_t i0 = ins0(k, a), i1 = i0 | ma;
        const C2 x = amp[i0], y = amp[i1];
        amp[i0] = C2{y.im, -y.re};
        amp[i1] = C2{-x.im, x.re};
      }
      break;
    case G_S: case G_SDG: case G_Z: case G_T: case G_TDG: case G_RZ: {
      C2 ph;
      if (kind == G_S) ph = C2{0.0, 1.0};
      else if (kind == G_SDG) ph = C2{0.0, -1.0};
      else if (kind == G_Z) ph = C2{-1.0, 0.0};
      else if (kind == G_T) ph = C2{0.70710678118654752440, 0.70710678118654752440};
      else if (kind == G_TDG) ph = C2{0.70710678118654752440, -0.70710678118654752440};
      else {
        double sn, cs;
        sincos(theta, &sn, &cs);
        ph = C2{cs, sn};
      }
      for (uint32_t k = threadIdx.x; k < half; k += kSvBlock) {
        const uint32_t i1 = ins0(k, a) | ma;
        amp[i1] = cmul(amp[i1], ph);
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

__global__ __launch_bounds__(kSvBlock) void sv_kernel(const FragDev *__restrict__ fd, uint64_t v0,
                                                      double *__restrict__ dist) {
  extern __shared__ C2 amp[];
  const FragDev &F = *fd;
  const uint32_t m = F.m;
  const uint32_t N = 1u << m;
  const uint64_t v = v0 + blockIdx.x;
  for (uint32_t i = threadIdx.x; i < N; i += kSvBlock) amp[i] = C2{i == 0 ? 1.0 : 0.0, 0.0};
  __syncthreads();
  {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 1 || d == 0) continue;
      const uint32_t q = F.axis_local[j];
      if (d == 1) {
        apply_gate(amp, m, G_X, q, 0, 0.0);
      } else {
        apply_gate(amp, m, G_H, q, 0, 0.0);
        if (d == 3) apply_gate(amp, m, G_S, q, 0, 0.0);
      }
    }
  }
  for (uint32_t g = 0; g < F.n_ops; ++g) {
    const uint32_t w = F.ops[g];
    apply_gate(amp, m, op_kind(w), op_q0(w), op_q1(w), F.theta ? F.theta[g] : 0.0);
  }
  {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 0 || d == 2) continue;
      const uint32_t q = F.axis_local[j];
      if (d == 1) apply_gate(amp, m, G_SDG, q, 0, 0.0);
      apply_gate(amp, m, G_H, q, 0, 0.0);
    }
  }
  // marginal over the measured set
  const uint32_t nm = F.n_meas;
  uint32_t mmask = 0;
  for (uint32_t j = 0; j < nm; ++j) mmask |= 1u << F.meas[j];
  const uint32_t rest = m - nm;
  double *out = dist + (uint64_t)blockIdx.x * (1ull << nm);
  for (uint32_t o = threadIdx.x; o < (1u << nm); o += kSvBlock) {
    uint32_t base = 0;
    for (uint32_t j = 0; j < nm; ++j) base |= ((o >> j) & 1u) << F.meas[j];
    double acc = 0.0;
    for (uint32_t r = 0; r < (1u << rest); ++r) {
      // scatter r into the unmeasured bit positions, ascending
      uint32_t idx = base, rr = r;
      for (uint32_t q = 0; q < m; ++q) {
        if (mmask & (1u << q)) continue;
        idx |= (rr & 1u) << q;
        rr >>= 1;
      }
      const C2 a = amp[idx];
      acc += a.re * a.re + a.im * a.im;
    }
    out[o] = acc;
  }
}

}  // namespace

hipError_t launch_sv(const FragDev *d_frag, const FragDev &h, uint64_t v0, uint64_t nv, double *dist,
                     hipStream_t s) {
  if (h.m > (uint32_t)kMaxNcQubits || h.n_meas > h.m) return hipErrorInvalidValue;
  const size_t lds = (size_t(1) << h.m) * sizeof(C2);
  hipError_t e = hipFuncSetAttribute((const void *)sv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  for (uint64_t done = 0; done < nv;) {
    uint64_t chunk = nv - done;
    if (chunk > (1ull << 30)) chunk = 1ull << 30;
    hipLaunchKernelGGL(sv_kernel, dim3((unsigned)chunk), dim3(kSvBlock), lds, s, d_frag, v0 + done,
                       dist + (done << h.n_meas));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

}  // namespace ccut
