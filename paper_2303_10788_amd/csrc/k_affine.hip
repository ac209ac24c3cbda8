// Affine sample models of Clifford fragment variants, read off in the
// Heisenberg picture instead of replaying the measurements on a tableau.
//
// A variant prepares a product stabilizer state (|0> on circuit inputs, its
// preparation on each quantum input), applies the fragment's Clifford U and
// measures the observables O_j (Z on a requested output, the basis Pauli X,
// Y or Z on a quantum output) in measured order.  Pulled back,
// Q_j = U^dag O_j U are commuting Paulis measured on the product state.  The
// stabilizer measurement sequence (Aaronson-Gottesman, the Clifford backend
// of Sec. V-B) gives: measurement j is deterministic iff some product
// prod_{k in c} Q_k with max(c) = j lies in the state's stabilizer group
// (up to sign), and then sum_{k in c} x_k = s(c), the sign of that product
// on the state; otherwise its outcome is a fresh random bit.  A Pauli is in
// the group of a product state iff on each qubit it is I or that qubit's
// stabilizer (Z for |0>, |1>; X for |+>; Y for |+i>), i.e. iff its
// "constraint vector" (x on Z-qubits, z on X-qubits, x ^ z on Y-qubits)
// is zero.  So measurement order Gaussian elimination of the constraint
// vectors gives, per measurement, either a pivot (random) or a combination
// c (deterministic) with its sign; resolving the relations in order gives
// each outcome as an affine function of the random bits: exactly the
// model (x0, randmask, G) the per-shot tableau simulation samples from.
//
// One wavefront per variant, lane j holding measurement j (at most 64):
// its Pauli Q_j (tracked as i^a X^x Z^z), its constraint vector, and the
// combination mask of the measurements folded into it.  Elimination is
// n_meas broadcast steps (readlane), no LDS and no barrier.
#include "common.hpp"

namespace ccut {

namespace {

__device__ inline uint64_t readlane64(uint64_t v, uint32_t lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// rows: the fragment's carried-back Hermitian Paulis U^dag P U in measured
// order (a requested output: its Z; a quantum output: its X, then its Z),
// each x[W], z[W], sign word; out: the variant's model words.
template <int W>
__device__ void affine_variant(const FragDev &F, const uint64_t *__restrict__ rows, uint64_t v,
                               uint64_t *__restrict__ out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n = F.n_meas;
  const bool live = lane < n;
  const uint32_t my_q = live ? (uint32_t)F.meas[lane] : 0xFFFFFFFFu;
  // the variant's preparations (stabilizer of each input qubit: Z with sign
  // for |0>, |1>; X for |+>; Y for |+i>) and this lane's basis digit
  uint64_t one[W], px[W], py[W];
#pragma unroll
  for (int w = 0; w < W; ++w) one[w] = px[w] = py[w] = 0;
  bool is_out = false;
  uint32_t bdig = 2;
  {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t radix = F.axis_radix[j];
      const uint32_t d = (uint32_t)(t % radix);
      t /= radix;
      const uint32_t q = F.axis_local[j];
      if (F.axis_side[j] == 1) {
        const uint64_t bit = 1ull << (q & 63);
#pragma unroll
        for (int w = 0; w < W; ++w)
          if ((q >> 6) == (uint32_t)w) {
            if (d == 1) one[w] |= bit;
            if (d == 2) px[w] |= bit;
            if (d == 3) py[w] |= bit;
          }
      } else if (q == my_q) {
        is_out = true;
        bdig = d;  // X 0, Y 1, Z 2
      }
    }
  }
  // this lane's row: every quantum output before it takes two rows
  const uint64_t outs = __ballot(is_out);
  const uint32_t r0 = lane + (uint32_t)__popcll(outs & ((1ull << lane) - 1ull));
  constexpr uint32_t RS = 2 * W + 1;
  uint64_t x[W], z[W];
  uint32_t a = 0;
  if (live) {
    const uint64_t *R = rows + (size_t)r0 * RS;
    if (is_out && bdig != 2) {
      // X row (basis X), or Y = i X Z from the X and Z rows (basis Y)
      uint32_t pr = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        x[w] = R[w];
        z[w] = R[W + w];
        pr += __popcll(x[w] & z[w]);
      }
      a = (2u * ((uint32_t)R[2 * W] & 1u) + pr) & 3u;
      if (bdig == 1) {
        const uint64_t *Q = R + RS;
        uint32_t cross = 0, pq = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          cross += __popcll(z[w] & Q[w]);
          pq += __popcll(Q[w] & Q[W + w]);
        }
        a = (a + 1u + 2u * ((uint32_t)Q[2 * W] & 1u) + pq + 2u * cross) & 3u;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          x[w] ^= Q[w];
          z[w] ^= Q[W + w];
        }
      }
    } else {
      const uint64_t *Q = R + (is_out ? RS : 0);  // a quantum output in Z: its Z row
      uint32_t pr = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        x[w] = Q[w];
        z[w] = Q[W + w];
        pr += __popcll(x[w] & z[w]);
      }
      a = (2u * ((uint32_t)Q[2 * W] & 1u) + pr) & 3u;
    }
  } else {
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = z[w] = 0;
  }
  uint64_t col[W];
#pragma unroll
  for (int w = 0; w < W; ++w) col[w] = (x[w] & ~(px[w] | py[w])) | (z[w] & px[w]) | ((x[w] ^ z[w]) & py[w]);
  uint64_t rec = live ? 1ull << lane : 0ull;
  bool det = false;
  // elimination in measurement order
  for (uint32_t j = 0; j < n; ++j) {
    uint64_t c[W], nz = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      c[w] = readlane64(col[w], j);
      nz |= c[w];
    }
    if (nz == 0) {
      det |= lane == j;
      continue;
    }
    // pivot: the lowest set bit of measurement j's vector (uniform)
    uint32_t pw = 0;
    uint64_t pb = 0;
#pragma unroll
    for (int w = W - 1; w >= 0; --w)
      if (c[w]) {
        pw = (uint32_t)w;
        pb = c[w] & (0ull - c[w]);
      }
    uint64_t cw = col[0];
#pragma unroll
    for (int w = 1; w < W; ++w)
      if (pw == (uint32_t)w) cw = col[w];
    const bool hit = live && lane > j && (cw & pb);
    uint64_t jx[W], jz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      jx[w] = readlane64(x[w], j);
      jz[w] = readlane64(z[w], j);
    }
    const uint32_t ja = __builtin_amdgcn_readlane(a, j);
    const uint64_t jrec = readlane64(rec, j);
    if (hit) {
      uint32_t cross = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) cross += __popcll(z[w] & jx[w]);
      a = (a + ja + 2u * cross) & 3u;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        col[w] ^= c[w];
        x[w] ^= jx[w];
        z[w] ^= jz[w];
      }
      rec ^= jrec;
    }
  }
  // sign of a deterministic measurement's product on the product state:
  // i^a times (-1) per |1> qubit with z = 1 and (-i) per |+i> qubit with
  // x = z = 1 (X Z = -i Y); the result is +1 or -1
  uint32_t cst = 0;
  if (det) {
    uint32_t ny = 0, n1 = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      ny += __popcll(x[w] & z[w] & py[w]);
      n1 += __popcll(z[w] & one[w]);
    }
    cst = ((a + 3u * ny + 2u * n1) & 3u) >> 1;
  }
  // outcome forms in measurement order: a random outcome is its own bit; a
  // deterministic one is its sign plus the earlier outcomes of its product
  uint64_t form = (live && !det) ? 1ull << lane : 0ull;
  for (uint32_t j = 0; j + 1 < n; ++j) {
    const uint64_t fj = readlane64(form, j);
    const uint32_t cj = __builtin_amdgcn_readlane(cst, j);
    if (det && lane > j && ((rec >> j) & 1ull)) {
      form ^= fj;
      cst ^= cj;
    }
  }
  const uint64_t x0 = __ballot(live && det && cst);
  const uint64_t rmask = __ballot(live && !det);
  uint64_t mycol = 0;
  for (uint32_t c2 = 0; c2 < n; ++c2) {
    const uint64_t g = __ballot(live && ((form >> c2) & 1ull));
    if (lane == c2) mycol = g;
  }
  if (lane == 0) {
    out[0] = x0;
    out[1] = rmask;
  }
  if (live) out[2 + lane] = mycol;
}

__device__ inline void affine_dispatch(uint32_t W, const FragDev &F, const uint64_t *rows, uint64_t v, uint64_t *out) {
  switch (W) {
    case 1: affine_variant<1>(F, rows, v, out); break;
    case 2: affine_variant<2>(F, rows, v, out); break;
    case 4: affine_variant<4>(F, rows, v, out); break;
    default: affine_variant<8>(F, rows, v, out); break;
  }
}

// Variants [v0, v0 + nv) of one fragment, one wave each.  vmask
// (optional, indexed by variant): variants with vmask[v] == 0 get no model
// (their shots are never drawn).
__global__ __launch_bounds__(256) void affine_kernel(const FragDev F, uint32_t W, const uint64_t *__restrict__ rows,
                                                     uint64_t v0, uint64_t nv, uint64_t *__restrict__ models,
                                                     const uint8_t *__restrict__ vmask) {
  const uint64_t i = (uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= nv) return;  // whole waves leave together
  if (vmask && !vmask[v0 + i]) return;
  affine_dispatch(W, F, rows, v0 + i, models + i * model_words(F.n_meas));
}

// Every Clifford variant of a batch: wave g takes items g, g + waves, ...
// (items sorted by cost, longest first); the fragment's row width is in the
// descriptor list (rows_off = word offset of its carried-back rows).
__global__ __launch_bounds__(1024) void affine_batch_kernel(const FragDev *__restrict__ descs,
                                                            const uint32_t *__restrict__ desc_w,
                                                            const BatchItem *__restrict__ items, uint32_t n_items,
                                                            const uint64_t *__restrict__ rows,
                                                            uint64_t *__restrict__ models) {
  const uint32_t waves = gridDim.x * (blockDim.x / 64);
  for (uint32_t i = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < n_items; i += waves) {
    const uint32_t idx = __builtin_amdgcn_readfirstlane(i);
    const BatchItem &it = items[idx];
    const uint32_t d = __builtin_amdgcn_readfirstlane(it.desc);
    affine_dispatch(desc_w[d], descs[d], rows + it.base_off, it.variant, models + it.model_off);
  }
}

// More than 64 measurements: one workgroup per variant, wave t's lane l
// holding measurement 64 t + l (meas_axis[j]: the axis of a quantum output,
// else -1; row_of[j]: its first carried-back row).  The elimination is the
// same, each step's pivot measurement broadcast through LDS (double
// buffered: one barrier per step).  The combination of a deterministic
// measurement holds itself and random measurements only (only pivots are
// ever folded into another vector), so its outcome is its sign plus the
// random outcomes of the rest of its combination: G[a] (the outcomes that
// random bit a flips) is a itself plus every deterministic j whose
// combination holds a.  Model: x0[MW], rmask[MW], G[a][MW] for a < n.
template <int W, int MW>
__global__ __launch_bounds__(1024) void affine_wide_kernel(const FragDev F, const int8_t *__restrict__ meas_axis,
                                                           const uint16_t *__restrict__ row_of, uint32_t n,
                                                           const uint64_t *__restrict__ rows, uint64_t v0,
                                                           uint64_t *__restrict__ models) {
  struct Bcast {
    uint64_t c[W], x[W], z[W], rec[MW];
    uint32_t a;
  };
  __shared__ Bcast s_b[2];
  const uint32_t me = threadIdx.x, lane = me & 63u, wave = me >> 6;
  const bool live = me < n;
  const uint64_t v = v0 + blockIdx.x;
  uint64_t *out = models + blockIdx.x * (uint64_t)model_words(n);
  uint64_t one[W], px[W], py[W];
#pragma unroll
  for (int w = 0; w < W; ++w) one[w] = px[w] = py[w] = 0;
  const int my_axis = live ? (int)meas_axis[me] : -1;
  bool is_out = my_axis >= 0;
  uint32_t bdig = 2;
  {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t radix = F.axis_radix[j];
      const uint32_t d = (uint32_t)(t % radix);
      t /= radix;
      const uint32_t q = F.axis_local[j];
      if (F.axis_side[j] == 1) {
        const uint64_t bit = 1ull << (q & 63);
#pragma unroll
        for (int w = 0; w < W; ++w)
          if ((q >> 6) == (uint32_t)w) {
            if (d == 1) one[w] |= bit;
            if (d == 2) px[w] |= bit;
            if (d == 3) py[w] |= bit;
          }
      } else if ((int)j == my_axis) {
        bdig = d;  // X 0, Y 1, Z 2
      }
    }
  }
  constexpr uint32_t RS = 2 * W + 1;
  uint64_t x[W], z[W];
  uint32_t a = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) x[w] = z[w] = 0;
  if (live) {
    const uint64_t *R = rows + (size_t)row_of[me] * RS;
    const uint64_t *Q = (is_out && bdig == 2) ? R + RS : R;  // a quantum output in Z: its Z row
    uint32_t pr = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      x[w] = Q[w];
      z[w] = Q[W + w];
      pr += __popcll(x[w] & z[w]);
    }
    a = (2u * ((uint32_t)Q[2 * W] & 1u) + pr) & 3u;
    if (is_out && bdig == 1) {  // Y = i X Z from the X and Z rows
      const uint64_t *Z = R + RS;
      uint32_t cross = 0, pq = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        cross += __popcll(z[w] & Z[w]);
        pq += __popcll(Z[w] & Z[W + w]);
      }
      a = (a + 1u + 2u * ((uint32_t)Z[2 * W] & 1u) + pq + 2u * cross) & 3u;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        x[w] ^= Z[w];
        z[w] ^= Z[W + w];
      }
    }
  }
  uint64_t col[W], rec[MW];
#pragma unroll
  for (int w = 0; w < W; ++w) col[w] = (x[w] & ~(px[w] | py[w])) | (z[w] & px[w]) | ((x[w] ^ z[w]) & py[w]);
#pragma unroll
  for (int w = 0; w < MW; ++w) rec[w] = (live && (me >> 6) == (uint32_t)w) ? 1ull << lane : 0ull;
  bool det = false;
  for (uint32_t j = 0; j < n; ++j) {
    Bcast &B = s_b[j & 1];
    if (me == j) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        B.c[w] = col[w];
        B.x[w] = x[w];
        B.z[w] = z[w];
      }
#pragma unroll
      for (int w = 0; w < MW; ++w) B.rec[w] = rec[w];
      B.a = a;
    }
    __syncthreads();
    uint64_t c[W], nz = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      c[w] = B.c[w];
      nz |= c[w];
    }
    if (nz == 0) {  // uniform: measurement j is deterministic
      det |= me == j;
      continue;
    }
    uint32_t pw = 0;
    uint64_t pb = 0;
#pragma unroll
    for (int w = W - 1; w >= 0; --w)
      if (c[w]) {
        pw = (uint32_t)w;
        pb = c[w] & (0ull - c[w]);
      }
    uint64_t cw = col[0];
#pragma unroll
    for (int w = 1; w < W; ++w)
      if (pw == (uint32_t)w) cw = col[w];
    if (live && me > j && (cw & pb)) {
      uint32_t cross = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) cross += __popcll(z[w] & B.x[w]);
      a = (a + B.a + 2u * cross) & 3u;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        col[w] ^= c[w];
        x[w] ^= B.x[w];
        z[w] ^= B.z[w];
      }
#pragma unroll
      for (int w = 0; w < MW; ++w) rec[w] ^= B.rec[w];
    }
  }
  uint32_t cst = 0;
  if (det) {
    uint32_t ny = 0, n1 = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      ny += __popcll(x[w] & z[w] & py[w]);
      n1 += __popcll(z[w] & one[w]);
    }
    cst = ((a + 3u * ny + 2u * n1) & 3u) >> 1;
  }
  // wave t writes word t of every model vector
  const uint64_t x0 = __ballot(live && det && cst);
  const uint64_t rmask = __ballot(live && !det);
  if (lane == 0 && wave < (uint32_t)MW) {
    out[wave] = x0;
    out[MW + wave] = rmask;
  }
  for (uint32_t aa = 0; aa < n; ++aa) {
    uint64_t rw = rec[0];
#pragma unroll
    for (int w = 1; w < MW; ++w)
      if ((aa >> 6) == (uint32_t)w) rw = rec[w];
    const bool bit = live && (me == aa ? !det : (det && ((rw >> (aa & 63)) & 1ull)));
    const uint64_t g = __ballot(bit);
    if (lane == 0 && wave < (uint32_t)MW) out[2 * MW + (uint64_t)aa * MW + wave] = g;
  }
  // words of waves beyond the measurements (MW rounded up): zero
  if (lane == 0)
    for (uint32_t w = (n + 63) / 64 + wave; w < (uint32_t)MW; w += blockDim.x / 64) {
      out[w] = 0;
      out[MW + w] = 0;
      for (uint32_t aa = 0; aa < n; ++aa) out[2 * MW + (uint64_t)aa * MW + w] = 0;
    }
}

}  // namespace

hipError_t launch_affine_wide(const FragDev &F, uint32_t W, const int8_t *meas_axis, const uint16_t *row_of,
                              uint32_t n_meas, const uint64_t *rows, uint64_t v0, uint64_t nv, uint64_t *models,
                              hipStream_t s) {
  if (nv == 0) return hipSuccess;
  const uint32_t MW = model_mw(n_meas);
  if (n_meas > (uint32_t)kMaxMeasWide || (W != 1 && W != 2 && W != 4 && W != 8) || F.m > 64 * W ||
      nv > 0x7FFFFFFFull)
    return hipErrorInvalidValue;
  const dim3 g((unsigned)nv), b(64 * ((n_meas + 63) / 64));
#define CCUT_AFFINE_WIDE(WW, MM) \
  hipLaunchKernelGGL((affine_wide_kernel<WW, MM>), g, b, 0, s, F, meas_axis, row_of, n_meas, rows, v0, models)
#define CCUT_AFFINE_WIDE_W(MM)          \
  switch (W) {                          \
    case 1: CCUT_AFFINE_WIDE(1, MM); break; \
    case 2: CCUT_AFFINE_WIDE(2, MM); break; \
    case 4: CCUT_AFFINE_WIDE(4, MM); break; \
    default: CCUT_AFFINE_WIDE(8, MM); break; \
  }
  switch (MW) {
    case 1: CCUT_AFFINE_WIDE_W(1); break;
    case 2: CCUT_AFFINE_WIDE_W(2); break;
    case 4: CCUT_AFFINE_WIDE_W(4); break;
    case 8: CCUT_AFFINE_WIDE_W(8); break;
    default: CCUT_AFFINE_WIDE_W(16); break;
  }
#undef CCUT_AFFINE_WIDE_W
#undef CCUT_AFFINE_WIDE
  return hipGetLastError();
}

hipError_t launch_affine(const FragDev &F, uint32_t W, const uint64_t *rows, uint64_t v0, uint64_t nv,
                         uint64_t *models, hipStream_t s, const uint8_t *vmask) {
  if (nv == 0) return hipSuccess;
  if (F.n_meas > (uint32_t)kMaxMeas || (W != 1 && W != 2 && W != 4 && W != 8) || F.m > 64 * W)
    return hipErrorInvalidValue;
  const uint64_t blocks = (nv + 3) / 4;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(affine_kernel, dim3((unsigned)blocks), dim3(256), 0, s, F, W, rows, v0, nv, models, vmask);
  return hipGetLastError();
}

hipError_t launch_affine_batch(const FragDev *descs, const uint32_t *desc_w, const BatchItem *items, uint32_t n_items,
                               const uint64_t *rows, uint64_t *models, uint32_t block, uint32_t grid, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  if (block % 64 || block == 0 || block > 1024 || grid == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(affine_batch_kernel, dim3(grid), dim3(block), 0, s, descs, desc_w, items, n_items, rows, models);
  return hipGetLastError();
}

}  // namespace ccut
