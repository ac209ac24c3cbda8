// Maximum-likelihood fragment correction (Sec. V-C, distribution builder:
// the fragment models are made self-consistent before the contraction).
//
// For one preparation combination s of a fragment's quantum inputs, the
// model is the set of conditional states {rho_x} of its n quantum outputs
// (d = 2^n) jointly with the outcome x of its requested outputs:
// p(o, x | s, b) = Tr(Pi_{b,o} rho_x) for basis combination b and outcome o
// on the quantum outputs.  The raw model is the least-squares inversion of
// the variant tables (each Pauli coefficient Tr(sigma_P rho_x) the mean of
// the parity estimates of every basis combination that measures P); the
// corrected model is the physical one (every rho_x positive semidefinite,
// sum_x Tr rho_x = 1) nearest to it in the Frobenius norm, the
// maximum-likelihood model under Gaussian noise: the blocks are
// diagonalised and their joint spectrum is projected onto the probability
// simplex with the eigenvectors kept.  The tables are then rewritten in
// place as the corrected model's probabilities, so the Pauli-basis
// transform and the contraction that follow are unchanged.
//
// Three launches per fragment:
//  1. one thread per (s, x): gather the 3^n x d table entries, form rho_x,
//     diagonalise it (cyclic complex Jacobi in registers), store the
//     eigenvalues;
//  2. one workgroup per s: the simplex shift tau_s of the joint spectrum by
//     Michelot's iteration (tau = (sum of the active values - 1) / their
//     count, active = the values above the previous tau, until the active
//     set stops shrinking), sums in a fixed order;
//  3. one thread per (s, x): the same diagonalisation again (the same code
//     on the same data: the same bits), eigenvalues max(mu - tau_s, 0),
//     rho'_x, its Pauli coefficients, the corrected table entries.
#include <cmath>

#include "common.hpp"

#pragma clang fp contract(off)

namespace ccut {

namespace {

struct Cx {
  double re, im;
};
__device__ inline Cx cx(double r, double i = 0.0) { return Cx{r, i}; }
__device__ inline Cx add(Cx a, Cx b) { return Cx{a.re + b.re, a.im + b.im}; }
__device__ inline Cx mul(Cx a, Cx b) { return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cx cnj(Cx a) { return Cx{a.re, -a.im}; }
__device__ inline Cx scl(Cx a, double s) { return Cx{a.re * s, a.im * s}; }

// The table index of outcome o on the quantum outputs and x on the
// requested outputs.
__device__ inline uint64_t ml_col(const MlJob &J, uint32_t o, uint64_t x) {
  uint64_t idx = 0;
  for (uint32_t i = 0; i < J.n_out; ++i) idx |= (uint64_t)((o >> i) & 1u) << J.opos[i];
  for (uint32_t i = 0; i < J.n_req; ++i) idx |= ((x >> i) & 1ull) << J.xpos[i];
  return idx;
}

// The variant index of preparation combination s (base 4, input axis 0
// least significant) and basis combination b (base 3, output 0 least
// significant).
__device__ inline uint64_t ml_row(const MlJob &J, uint32_t s, uint32_t b) {
  uint64_t v = 0;
  for (uint32_t j = 0; j < J.n_in; ++j) v += (uint64_t)((s >> (2 * j)) & 3u) * J.istride[j];
  for (uint32_t i = 0; i < J.n_out; ++i) {
    v += (uint64_t)(b % 3) * J.ostride[i];
    b /= 3;
  }
  return v;
}

// Pauli letter of qubit i in P (base 4, qubit 0 least significant): 0 I,
// 1 X, 2 Y, 3 Z; the basis letters X, Y, Z are the Paulis 1, 2, 3.
// sigma_P = sigma_{P_0} (x) sigma_{P_1} (x) ..., qubit 0 the most
// significant index bit of the d x d matrix.  Row r of sigma_P has its one
// nonzero entry in column r ^ flip(P), with the phase below.
template <int N>
__device__ inline uint32_t pauli_flip(uint32_t P) {
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const uint32_t l = (P >> (2 * i)) & 3u;
    if (l == 1 || l == 2) m |= 1u << (N - 1 - i);
  }
  return m;
}
template <int N>
__device__ inline Cx pauli_phase(uint32_t P, uint32_t r) {
  Cx ph = cx(1.0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const uint32_t l = (P >> (2 * i)) & 3u, bit = (r >> (N - 1 - i)) & 1u;
    if (l == 2) ph = mul(ph, bit ? cx(0.0, 1.0) : cx(0.0, -1.0));  // Y: [[0, -i], [i, 0]]
    if (l == 3 && bit) ph = scl(ph, -1.0);                           // Z: [[1, 0], [0, -1]]
  }
  return ph;
}

// rho_x of thread (s, x) from the tables and its eigen-decomposition
// A = V diag(w) V^dagger (w in A's diagonal on return).
template <int N>
__device__ inline void ml_eigen(const MlJob &J, uint32_t s, uint64_t x, Cx (&A)[1 << N][1 << N],
                                Cx (&V)[1 << N][1 << N]) {
  constexpr int D = 1 << N, NB = N == 1 ? 3 : 9, NP = 1 << (2 * N);
  double p[NB][D];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const double *row = J.dist + ml_row(J, s, (uint32_t)b) * J.row_len;
#pragma unroll
    for (int o = 0; o < D; ++o) p[b][o] = row[ml_col(J, (uint32_t)o, x)];
  }
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      A[r][c] = cx(0.0);
      V[r][c] = cx(r == c ? 1.0 : 0.0);
    }
  // least-squares Pauli coefficients: the mean over compatible bases, in
  // ascending basis order, of sum_o (-1)^(o on P's support) p(o | b)
#pragma unroll
  for (int P = 0; P < NP; ++P) {
    double sum = 0.0;
    int cnt = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      bool ok = true;
      int bb = b;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = (P >> (2 * i)) & 3;
        if (l != 0 && l != bb % 3 + 1) ok = false;
        bb /= 3;
      }
      if (!ok) continue;
      double e = 0.0;
#pragma unroll
      for (int o = 0; o < D; ++o) {
        int par = 0;
#pragma unroll
        for (int i = 0; i < N; ++i)
          if ((P >> (2 * i)) & 3) par ^= (o >> i) & 1;
        e = par ? e - p[b][o] : e + p[b][o];
      }
      sum += e;
      ++cnt;
    }
    const double c = sum / cnt / D;
    const uint32_t fl = pauli_flip<N>((uint32_t)P);
#pragma unroll
    for (int r = 0; r < D; ++r) A[r][r ^ fl] = add(A[r][r ^ fl], scl(pauli_phase<N>((uint32_t)P, (uint32_t)r), c));
  }
  // cyclic Jacobi: rotations G = diag(1, e^{-i phi}) R(theta) on (p, q)
  // zero A_pq; A <- G^dagger A G, V <- V G
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = 0.0, diag = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      diag += A[r][r].re * A[r][r].re;
#pragma unroll
      for (int c = r + 1; c < D; ++c) off += A[r][c].re * A[r][c].re + A[r][c].im * A[r][c].im;
    }
    if (off <= 1e-34 * diag || off == 0.0) break;
#pragma unroll
    for (int pp = 0; pp < D; ++pp)
#pragma unroll
      for (int qq = pp + 1; qq < D; ++qq) {
        const Cx apq = A[pp][qq];
        const double r = sqrt(apq.re * apq.re + apq.im * apq.im);
        if (r == 0.0) continue;
        const Cx e = cx(apq.re / r, apq.im / r);  // e^{i phi}
        const double th = (A[qq][qq].re - A[pp][pp].re) / (2.0 * r);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        const Cx gpp = cx(c), gpq = cx(sn), gqp = scl(cnj(e), -sn), gqq = scl(cnj(e), c);
#pragma unroll
        for (int k = 0; k < D; ++k) {  // columns: A G, V G
          const Cx akp = A[k][pp], akq = A[k][qq];
          A[k][pp] = add(mul(akp, gpp), mul(akq, gqp));
          A[k][qq] = add(mul(akp, gpq), mul(akq, gqq));
          const Cx vkp = V[k][pp], vkq = V[k][qq];
          V[k][pp] = add(mul(vkp, gpp), mul(vkq, gqp));
          V[k][qq] = add(mul(vkp, gpq), mul(vkq, gqq));
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {  // rows: G^dagger (A G)
          const Cx apk = A[pp][k], aqk = A[qq][k];
          A[pp][k] = add(mul(cnj(gpp), apk), mul(cnj(gqp), aqk));
          A[qq][k] = add(mul(cnj(gpq), apk), mul(cnj(gqq), aqk));
        }
        A[pp][qq] = A[qq][pp] = cx(0.0);
        A[pp][pp].im = A[qq][qq].im = 0.0;
      }
  }
}

template <int N>
__global__ __launch_bounds__(256) void ml_block_kernel(const MlJob *__restrict__ jp, uint32_t phase) {
  const MlJob &J = *jp;
  constexpr int D = 1 << N, NB = N == 1 ? 3 : 9, NP = 1 << (2 * N);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)J.n_prep * J.nx) return;
  const uint32_t s = (uint32_t)(t / J.nx);
  const uint64_t x = t % J.nx;
  Cx A[D][D], V[D][D];
  ml_eigen<N>(J, s, x, A, V);
  if (phase == 0) {
#pragma unroll
    for (int k = 0; k < D; ++k) J.eig[t * D + k] = A[k][k].re;
    return;
  }
  const double tau = J.tau[s];
  double lam[D];
#pragma unroll
  for (int k = 0; k < D; ++k) lam[k] = fmax(A[k][k].re - tau, 0.0);
  // rho' = V diag(lam) V^dagger
  Cx R[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      Cx acc = cx(0.0);
#pragma unroll
      for (int k = 0; k < D; ++k) acc = add(acc, scl(mul(V[r][k], cnj(V[c][k])), lam[k]));
      R[r][c] = acc;
    }
  // Pauli coefficients Tr(sigma_P rho') = sum_r phase(P, r) rho'[r ^ flip][r]
  double cp[NP];
#pragma unroll
  for (int P = 0; P < NP; ++P) {
    const uint32_t fl = pauli_flip<N>((uint32_t)P);
    Cx acc = cx(0.0);
#pragma unroll
    for (int r = 0; r < D; ++r) acc = add(acc, mul(pauli_phase<N>((uint32_t)P, (uint32_t)r), R[r ^ fl][r]));
    cp[P] = acc.re;
  }
  // p'(o | b) = 2^-n sum over P measured by b of (-1)^(o on P's support) c'_P
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double *row = J.dist + ml_row(J, s, (uint32_t)b) * J.row_len;
#pragma unroll
    for (int o = 0; o < D; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int P = 0; P < NP; ++P) {
        bool ok = true;
        int bb = b, par = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const int l = (P >> (2 * i)) & 3;
          if (l != 0 && l != bb % 3 + 1) ok = false;
          if (l != 0) par ^= (o >> i) & 1;
          bb /= 3;
        }
        if (ok) acc = par ? acc - cp[P] : acc + cp[P];
      }
      row[ml_col(J, (uint32_t)o, x)] = acc / D;
    }
  }
}

// One workgroup per preparation combination: the simplex shift of its
// n = nx d eigenvalues (Michelot's iteration; fixed-order sums).
constexpr uint32_t kTauThreads = 256;
__global__ __launch_bounds__(kTauThreads) void ml_tau_kernel(const MlJob *__restrict__ jp, uint32_t d) {
  const MlJob &J = *jp;
  __shared__ double s_sum[kTauThreads];
  __shared__ uint64_t s_cnt[kTauThreads];
  const uint32_t s = blockIdx.x, tid = threadIdx.x;
  const uint64_t n = J.nx * d;
  const double *mu = J.eig + (uint64_t)s * n;
  // the active set starts as every value: tau below all of them
  double tau = -INFINITY;
  uint64_t prev = n + 1;
  for (;;) {
    double sum = 0.0;
    uint64_t cnt = 0;
    for (uint64_t i = tid; i < n; i += kTauThreads)
      if (mu[i] > tau) {
        sum += mu[i];
        ++cnt;
      }
    s_sum[tid] = sum;
    s_cnt[tid] = cnt;
    __syncthreads();
    for (uint32_t h = kTauThreads / 2; h; h >>= 1) {
      if (tid < h) {
        s_sum[tid] += s_sum[tid + h];
        s_cnt[tid] += s_cnt[tid + h];
      }
      __syncthreads();
    }
    const double tot = s_sum[0];
    const uint64_t c = s_cnt[0];
    __syncthreads();  // every thread has read the totals
    if (c == prev || c == 0) break;  // the active set stopped shrinking (c >= 1 always)
    tau = (tot - 1.0) / (double)c;
    prev = c;
  }
  if (tid == 0) J.tau[s] = tau;
}

}  // namespace

hipError_t launch_ml_correct(const MlJob &h, const MlJob *d_job, hipStream_t s) {
  const uint64_t threads = (uint64_t)h.n_prep * h.nx;
  if (threads == 0) return hipSuccess;
  if (h.n_out < 1 || h.n_out > 2) return hipErrorInvalidValue;
  const uint64_t blocks = (threads + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const uint32_t d = 1u << h.n_out;
  for (uint32_t phase = 0; phase < 2; ++phase) {
    if (h.n_out == 1)
      hipLaunchKernelGGL(ml_block_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, d_job, phase);
    else
      hipLaunchKernelGGL(ml_block_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, d_job, phase);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (phase == 0) {
      hipLaunchKernelGGL(ml_tau_kernel, dim3(h.n_prep), dim3(kTauThreads), 0, s, d_job, d);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace ccut
