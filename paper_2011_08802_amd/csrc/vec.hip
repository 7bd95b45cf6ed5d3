// Vector kernels: FGMRES reductions (wavefront shuffles + LDS, two-stage,
// deterministic), layout conversions, boundary conditions, state updates.
#include "common.h"

namespace mvpf {

constexpr int RB = 256;  // reduction block size

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;  // valid in thread 0
}

int red_blocks(int64_t n) {
  const int64_t b = (n + 1023) / 1024;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, MAX_RED_BLOCKS));
}

// part[j * nblk + blk] = sum over the block's chunk of V_j . w, j < k.
// The vectors are taken MD_G at a time, so w is read once per group (not
// once per vector), and the group's MD_G block sums share one barrier.
constexpr int MD_G = 8;
constexpr int MD_U = 4;
__device__ __forceinline__ void multidot_body(int64_t n, const double* __restrict__ V, int64_t ldv, int k,
                                              const double* __restrict__ w, double* __restrict__ part, int bid,
                                              int nblk) {
  __shared__ double sh[MD_G][RB / 64];
  const int64_t chunk = (n + nblk - 1) / nblk;
  const int64_t lo = (int64_t)bid * chunk;
  const int64_t hi = std::min<int64_t>(n, lo + chunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j0 = 0; j0 < k; j0 += MD_G) {
    const int g_n = std::min(MD_G, k - j0);  // uniform
    double s[MD_G];
#pragma unroll
    for (int g = 0; g < MD_G; ++g) s[g] = 0.0;
    const double* v0 = V + (int64_t)j0 * ldv;
    // MD_U rows per thread loaded together (one memory round trip instead of
    // MD_U), summed in the same order as one row at a time
    int64_t i = lo + threadIdx.x;
    for (; i + (MD_U - 1) * RB < hi; i += MD_U * RB) {
      double wv[MD_U], vv[MD_U][MD_G];
#pragma unroll
      for (int u = 0; u < MD_U; ++u) wv[u] = w[i + u * RB];
#pragma unroll
      for (int u = 0; u < MD_U; ++u)
#pragma unroll
        for (int g = 0; g < MD_G; ++g) vv[u][g] = g < g_n ? v0[(int64_t)g * ldv + i + u * RB] : 0.0;
#pragma unroll
      for (int u = 0; u < MD_U; ++u)
#pragma unroll
        for (int g = 0; g < MD_G; ++g)
          if (g < g_n) s[g] += vv[u][g] * wv[u];
    }
    for (; i < hi; i += RB) {
      const double wi = w[i];
#pragma unroll
      for (int g = 0; g < MD_G; ++g)
        if (g < g_n) s[g] += v0[(int64_t)g * ldv + i] * wi;
    }
#pragma unroll
    for (int g = 0; g < MD_G; ++g) {
      double v = s[g];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) sh[g][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < g_n) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < RB / 64; ++q) t += sh[threadIdx.x][q];
      part[(int64_t)(j0 + threadIdx.x) * nblk + bid] = t;
    }
    __syncthreads();
  }
}
__global__ void __launch_bounds__(RB) multidot_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, int k,
                                                      const double* __restrict__ w, double* __restrict__ part) {
  multidot_body(n, V, ldv, k, w, part, blockIdx.x, gridDim.x);
}

void launch_multidot(int64_t n, const double* V, int64_t ldv, int k, const double* w, double* part, hipStream_t s) {
  multidot_kernel<<<red_blocks(n), RB, 0, s>>>(n, V, ldv, k, w, part);
}

// out[j] (+)= sum_b part[j * nblk + b]
__device__ __forceinline__ void reduce_body(int nblk, const double* __restrict__ part, double* __restrict__ out,
                                            int accumulate, int j) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RB) s += part[(int64_t)j * nblk + b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[j] = accumulate ? out[j] + s : s;
}
__global__ void __launch_bounds__(RB) reduce_kernel(int nblk, const double* __restrict__ part, double* __restrict__ out,
                                                    int accumulate) {
  reduce_body(nblk, part, out, accumulate, blockIdx.x);
}

void launch_reduce(int k, int nblk, const double* part, double* out, int accumulate, hipStream_t s) {
  reduce_kernel<<<k, RB, 0, s>>>(nblk, part, out, accumulate);
}

// w -= sum_j h_j V_j ; optional part_norm[blk] = sum of w^2 over the chunk
__device__ __forceinline__ void multiaxpy_body(int64_t n, const double* __restrict__ V, int64_t ldv, int k,
                                               const double* __restrict__ h, double* __restrict__ w,
                                               double* __restrict__ part_norm, int bid, int nblk) {
  __shared__ double sh[RB / 64];
  __shared__ double hs[MAX_RESTART + 2];
  for (int j = threadIdx.x; j < k; j += RB) hs[j] = h[j];
  __syncthreads();
  const int64_t chunk = (n + nblk - 1) / nblk;
  const int64_t lo = (int64_t)bid * chunk;
  const int64_t hi = std::min<int64_t>(n, lo + chunk);
  double nrm = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += RB) {
    double s = w[i];
    for (int j = 0; j < k; ++j) s -= hs[j] * V[(int64_t)j * ldv + i];
    w[i] = s;
    nrm += s * s;
  }
  if (part_norm) {
    nrm = block_sum(nrm, sh);
    if (threadIdx.x == 0) part_norm[bid] = nrm;
  }
}
__global__ void __launch_bounds__(RB) multiaxpy_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, int k,
                                                       const double* __restrict__ h, double* __restrict__ w,
                                                       double* __restrict__ part_norm) {
  multiaxpy_body(n, V, ldv, k, h, w, part_norm, blockIdx.x, gridDim.x);
}

// The same update with a row's k basis entries loaded together (k <= KB:
// up to 8 loads in flight instead of one); with KD > 0, also the projections
// of the updated w on the first min(k, KD) basis vectors, part[j * nblk + blk]
// = the chunk's sum of V_j . w (classical Gram-Schmidt: the first pass's
// update and the second pass's projections in one sweep over the basis);
// with KD = 0 and part, the chunk's sum of w^2.  Every thread takes the rows,
// and every sum its terms, in the order of multiaxpy_body and multidot_body,
// so the results are bitwise theirs.
template <int KB, int KD>
__global__ void __launch_bounds__(RB) multiaxpy_reg_kernel(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                           int k, const double* __restrict__ h,
                                                           double* __restrict__ w, double* __restrict__ part) {
  constexpr int NA = KD > 0 ? KD : 1;
  __shared__ double sh[NA][RB / 64];
  __shared__ double hs[KB];
  for (int j = threadIdx.x; j < k; j += RB) hs[j] = h[j];
  __syncthreads();
  const int bid = blockIdx.x, nblk = gridDim.x;
  const int64_t chunk = (n + nblk - 1) / nblk;
  const int64_t lo = (int64_t)bid * chunk;
  const int64_t hi = std::min<int64_t>(n, lo + chunk);
  double acc[NA];
#pragma unroll
  for (int g = 0; g < NA; ++g) acc[g] = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += RB) {
    double s = w[i];
    double keep[NA];  // the entries of the first KD vectors, for the projections
#pragma unroll
    for (int g0 = 0; g0 < KB; g0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = g0 + u < k ? V[(int64_t)(g0 + u) * ldv + i] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (g0 + u < k) s -= hs[g0 + u] * v[u];
      if constexpr (KD > 0) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (g0 + u < KD) keep[g0 + u] = v[u];
      }
    }
    w[i] = s;
    if constexpr (KD > 0) {
#pragma unroll
      for (int g = 0; g < KD; ++g)
        if (g < k) acc[g] += keep[g] * s;
    } else {
      acc[0] += s * s;
    }
  }
  if (!part) return;  // uniform
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if constexpr (KD > 0) {
    const int kd = std::min(k, KD);
#pragma unroll
    for (int g = 0; g < KD; ++g) {
      if (g < kd) {
        double v = acc[g];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sh[g][wid] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x < kd) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < RB / 64; ++q) t += sh[threadIdx.x][q];
      part[(int64_t)threadIdx.x * nblk + bid] = t;
    }
  } else {
    const double nrm = block_sum(acc[0], &sh[0][0]);
    if (threadIdx.x == 0) part[bid] = nrm;
  }
}

// register tiers k <= 8, 16, 24, 32 (false above), the projections on all k
// vectors from the kept entries (157 VGPRs at 24, 206 at 32, no spills;
// measured at 76.7 M entries against projections on the first 16 and
// multidot for the rest: 22 % faster at k = 24, 29 % at k = 31)
template <bool DOT>
bool launch_multiaxpy_reg(int64_t n, const double* V, int64_t ldv, int k, const double* h, double* w, double* part,
                          hipStream_t s) {
  const int nb = red_blocks(n);
  if (k <= 8)
    multiaxpy_reg_kernel<8, DOT ? 8 : 0><<<nb, RB, 0, s>>>(n, V, ldv, k, h, w, part);
  else if (k <= 16)
    multiaxpy_reg_kernel<16, DOT ? 16 : 0><<<nb, RB, 0, s>>>(n, V, ldv, k, h, w, part);
  else if (k <= 24)
    multiaxpy_reg_kernel<24, DOT ? 24 : 0><<<nb, RB, 0, s>>>(n, V, ldv, k, h, w, part);
  else if (k <= 32)
    multiaxpy_reg_kernel<32, DOT ? 32 : 0><<<nb, RB, 0, s>>>(n, V, ldv, k, h, w, part);
  else
    return false;
  return true;
}

void launch_multiaxpy(int64_t n, const double* V, int64_t ldv, int k, const double* h, double* w, double* part_norm,
                      hipStream_t s) {
  if (launch_multiaxpy_reg<false>(n, V, ldv, k, h, w, part_norm, s)) return;
  multiaxpy_kernel<<<red_blocks(n), RB, 0, s>>>(n, V, ldv, k, h, w, part_norm);
}

void launch_multiaxpy_dot(int64_t n, const double* V, int64_t ldv, int k, const double* h, double* w, double* part,
                          hipStream_t s) {
  if (launch_multiaxpy_reg<true>(n, V, ldv, k, h, w, part, s)) return;
  launch_multiaxpy(n, V, ldv, k, h, w, nullptr, s);
  multidot_kernel<<<red_blocks(n), RB, 0, s>>>(n, V, ldv, k, w, part);
}

__global__ void __launch_bounds__(RB) scale_kernel(int64_t n, const double* __restrict__ w, const double* beta,
                                                   double* __restrict__ v) {
  const double ib = 1.0 / beta[0];
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) v[i] = w[i] * ib;
}

void launch_scale(int64_t n, const double* w, const double* beta, double* v, hipStream_t s) {
  scale_kernel<<<1024, RB, 0, s>>>(n, w, beta, v);
}

// x += sum_j y_j Z_j
template <typename TZ>
__global__ void __launch_bounds__(RB) combine_kernel(int64_t n, const TZ* __restrict__ Z, int64_t ldz, int k,
                                                     const double* __restrict__ y, double* __restrict__ x) {
  __shared__ double ys[MAX_RESTART + 2];
  for (int j = threadIdx.x; j < k; j += RB) ys[j] = y[j];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    double s = x[i];
    for (int j = 0; j < k; ++j) s += ys[j] * (double)Z[(int64_t)j * ldz + i];
    x[i] = s;
  }
}

template <typename TZ>
void launch_combine(int64_t n, const TZ* Z, int64_t ldz, int k, const double* y, double* x, hipStream_t s) {
  combine_kernel<TZ><<<1024, RB, 0, s>>>(n, Z, ldz, k, y, x);
}
template void launch_combine<float>(int64_t, const float*, int64_t, int, const double*, double*, hipStream_t);
template void launch_combine<double>(int64_t, const double*, int64_t, int, const double*, double*, hipStream_t);

// z = a x + b y (y may be null when b == 0)
__global__ void __launch_bounds__(RB) axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                                                   const double* __restrict__ y, double* __restrict__ z) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB)
    z[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z, hipStream_t s) {
  axpby_kernel<<<1024, RB, 0, s>>>(n, a, x, b, y, z);
}

template <typename T>
__global__ void __launch_bounds__(RB) zero_kernel(int64_t n, T* p) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) p[i] = (T)0;
}

template <typename T>
void launch_zero(int64_t n, T* p, hipStream_t s) {
  zero_kernel<T><<<1024, RB, 0, s>>>(n, p);
}
template void launch_zero<float>(int64_t, float*, hipStream_t);
template void launch_zero<double>(int64_t, double*, hipStream_t);

// ---- layout conversions ---------------------------------------------------
// out[(comp0 + c) * Npad + n] = in[n * ldc + c], c < ncomp  (out is SoA)
__global__ void __launch_bounds__(RB) i2s_kernel(Grid g, const double* __restrict__ in, int ncomp, int comp0,
                                                 int ldc, double* __restrict__ out) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.Npad) return;
  for (int c = 0; c < ncomp; ++c)
    out[(int64_t)(comp0 + c) * g.Npad + n] = (n < g.N) ? in[(int64_t)n * ldc + c] : 0.0;
}

void launch_interleaved_to_soa(const Grid& g, const double* in, int ncomp, int comp0, int ldc, double* out,
                               hipStream_t s) {
  i2s_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, in, ncomp, comp0, ldc, out);
}

__global__ void __launch_bounds__(RB) s2i_kernel(Grid g, const double* __restrict__ in, int ncomp, int comp0,
                                                 int ldc, double* __restrict__ out) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.N) return;
  for (int c = 0; c < ncomp; ++c) out[(int64_t)n * ldc + c] = in[(int64_t)(comp0 + c) * g.Npad + n];
}

void launch_soa_to_interleaved(const Grid& g, const double* in, int ncomp, int comp0, int ldc, double* out,
                               hipStream_t s) {
  s2i_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, in, ncomp, comp0, ldc, out);
}

// out = in with constrained dofs (and padding) zeroed, converted to TO
template <typename TI, typename TO>
__device__ __forceinline__ void convert_masked_body(const Grid& g, const TI* __restrict__ in,
                                                    const uint16_t* __restrict__ mask, TO* __restrict__ out, int bid) {
  const int n = bid * RB + threadIdx.x;
  if (n >= g.Npad) return;
  const unsigned m = (n < g.N) ? mask[n] : (1u << NDOF) - 1u;
#pragma unroll
  for (int c = 0; c < NDOF; ++c)
    out[(int64_t)c * g.Npad + n] = ((m >> c) & 1) ? (TO)0 : (TO)in[(int64_t)c * g.Npad + n];
}
template <typename TI, typename TO>
__global__ void __launch_bounds__(RB) convert_masked_kernel(Grid g, const TI* __restrict__ in,
                                                            const uint16_t* __restrict__ mask, TO* __restrict__ out) {
  convert_masked_body<TI, TO>(g, in, mask, out, blockIdx.x);
}

template <typename TI, typename TO>
void launch_convert_masked(const Grid& g, const TI* in, const uint16_t* mask, TO* out, hipStream_t s) {
  convert_masked_kernel<TI, TO><<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, in, mask, out);
}
template void launch_convert_masked<double, float>(const Grid&, const double*, const uint16_t*, float*, hipStream_t);
template void launch_convert_masked<double, double>(const Grid&, const double*, const uint16_t*, double*,
                                                    hipStream_t);
template void launch_convert_masked<float, float>(const Grid&, const float*, const uint16_t*, float*, hipStream_t);
template void launch_convert_masked<float, double>(const Grid&, const float*, const uint16_t*, double*, hipStream_t);

// dst[c][n] = src[c][n] on constrained dofs (the preconditioner is the
// identity there); src FP64, dst FP64
__global__ void __launch_bounds__(RB) set_constrained_kernel(Grid g, const uint16_t* __restrict__ mask,
                                                             const double* __restrict__ src, double* __restrict__ dst) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.N) return;
  const unsigned m = mask[n];
  if (!m) return;
#pragma unroll
  for (int c = 0; c < NDOF; ++c)
    if ((m >> c) & 1) dst[(int64_t)c * g.Npad + n] = src[(int64_t)c * g.Npad + n];
}

void launch_set_constrained(const Grid& g, const uint16_t* mask, const double* src, double* dst, hipStream_t s) {
  set_constrained_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, mask, src, dst);
}

// ---- boundary conditions and Newton updates ---------------------------------
__global__ void __launch_bounds__(RB) dirichlet_masks_kernel(Grid g, int kind, int patch, double radius, double depth,
                                                             uint16_t* __restrict__ mask, double* __restrict__ target) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.Npad) return;
  unsigned m = 0;
  double t = 0.0;
  if (n < g.N) {
    const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
    if (k == 0) m |= 7u;                 // bottom face: u = 0
    if (k == g.nz) {                     // top face
      if (kind == MVPF_LOAD_PATCH) {
        const int hp = patch / 2;
        if (abs(i - g.nx / 2) <= hp && abs(j - g.ny / 2) <= hp) {
          m |= 4u;
          t = -depth;
        }
      } else if (kind == MVPF_LOAD_CAP) {
        const double x = i * g.h - 0.5 * g.nx * g.h, y = j * g.h - 0.5 * g.ny * g.h;
        const double r2 = x * x + y * y;
        if (r2 < 2.0 * radius * depth - depth * depth) {
          m |= 4u;
          t = -(depth - (radius - sqrt(radius * radius - r2)));
        }
      }
    }
  }
  mask[n] = (uint16_t)m;
  target[n] = t;
}

void launch_dirichlet_masks(const Grid& g, const mvpf_loading& ld, double depth, uint16_t* mask, double* target,
                            hipStream_t s) {
  dirichlet_masks_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, ld.kind, ld.patch, ld.radius, depth, mask, target);
}

// g = target - current on constrained displacement dofs, 0 elsewhere
__global__ void __launch_bounds__(RB) increment_kernel(Grid g, const uint16_t* __restrict__ mask,
                                                       const double* __restrict__ target,
                                                       const double* __restrict__ state, double* __restrict__ gv) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.Npad) return;
  const unsigned m = (n < g.N) ? mask[n] : 0;
#pragma unroll
  for (int c = 0; c < NDOF; ++c) {
    double v = 0.0;
    if ((m >> c) & 1) v = (c == 2 ? target[n] : 0.0) - state[(int64_t)c * g.Npad + n];
    gv[(int64_t)c * g.Npad + n] = v;
  }
}

void launch_increment(const Grid& g, const uint16_t* mask, const double* target, const double* state, double* gvec,
                      hipStream_t s) {
  increment_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, mask, target, state, gvec);
}

// rhs = g on constrained dofs, -R - K g elsewhere
__global__ void __launch_bounds__(RB) newton_rhs_kernel(Grid g, const uint16_t* __restrict__ mask,
                                                        const double* __restrict__ R, const double* __restrict__ Kg,
                                                        const double* __restrict__ gv, double* __restrict__ rhs) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.Npad) return;
  const unsigned m = (n < g.N) ? mask[n] : 0;
#pragma unroll
  for (int c = 0; c < NDOF; ++c) {
    const int64_t q = (int64_t)c * g.Npad + n;
    rhs[q] = (n >= g.N) ? 0.0 : (((m >> c) & 1) ? gv[q] : -R[q] - Kg[q]);
  }
}

void launch_newton_rhs(const Grid& g, const uint16_t* mask, const double* R, const double* Kg, const double* gvec,
                       double* rhs, hipStream_t s) {
  newton_rhs_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, mask, R, Kg, gvec, rhs);
}

// U <- U + dx on free dofs; constrained dofs set to their targets
__global__ void __launch_bounds__(RB) state_update_kernel(Grid g, const uint16_t* __restrict__ mask,
                                                          const double* __restrict__ target,
                                                          const double* __restrict__ dx, double* __restrict__ st) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.N) return;
  const unsigned m = mask[n];
#pragma unroll
  for (int c = 0; c < NDOF; ++c) {
    const int64_t q = (int64_t)c * g.Npad + n;
    st[q] = ((m >> c) & 1) ? (c == 2 ? target[n] : 0.0) : st[q] + dx[q];
  }
}

void launch_state_update(const Grid& g, const uint16_t* mask, const double* target, const double* dx, double* state,
                         hipStream_t s) {
  state_update_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, mask, target, dx, state);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(RB) init_random_kernel(Grid g, uint64_t seed, double* __restrict__ st) {
  const int n = blockIdx.x * RB + threadIdx.x;
  if (n >= g.Npad) return;
  for (int c = 0; c < 3; ++c) st[(int64_t)c * g.Npad + n] = 0.0;
  for (int i = 0; i < NV; ++i) {
    double v = 0.0;
    if (n < g.N) {
      const uint64_t r = splitmix64(seed ^ (uint64_t)((uint64_t)NDOF * (uint64_t)n + 3ull + (uint64_t)i));
      v = 0.05 * ((double)(r >> 11) * 0x1.0p-53);
    }
    st[(int64_t)(3 + i) * g.Npad + n] = v;
    st[(int64_t)(3 + NV + i) * g.Npad + n] = v;
  }
}

void launch_init_random(const Grid& g, uint64_t seed, double* state, hipStream_t s) {
  init_random_kernel<<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, seed, state);
}

__global__ void __launch_bounds__(RB) free_norm_kernel(Grid g, const double* __restrict__ v,
                                                       const uint16_t* __restrict__ mask, double* __restrict__ part) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int n = blockIdx.x * RB + threadIdx.x; n < g.N; n += gridDim.x * RB) {
    const unsigned m = mask[n];
#pragma unroll
    for (int c = 0; c < NDOF; ++c) {
      const double x = v[(int64_t)c * g.Npad + n];
      if (!((m >> c) & 1)) s += x * x;
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_free_norm_partial(const Grid& g, const double* v, const uint16_t* mask, double* part, hipStream_t s) {
  free_norm_kernel<<<red_blocks((int64_t)g.N * NDOF), RB, 0, s>>>(g, v, mask, part);
}

// flat type conversion out[i] = (TO) in[i]
template <typename TI, typename TO>
__global__ void __launch_bounds__(RB) convert_kernel(int64_t n, const TI* __restrict__ in, TO* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) out[i] = (TO)in[i];
}

template <typename TI, typename TO>
void launch_convert(int64_t n, const TI* in, TO* out, hipStream_t s) {
  convert_kernel<TI, TO><<<1024, RB, 0, s>>>(n, in, out);
}
template void launch_convert<float, double>(int64_t, const float*, double*, hipStream_t);
template void launch_convert<double, float>(int64_t, const double*, float*, hipStream_t);

// Preconditioner output: z = V-cycle result on free dofs, z = v on
// constrained dofs of the finest level (identity there).
template <typename T, typename TZ>
__device__ __forceinline__ void precond_finish_body(const Grid& g, const T* __restrict__ x,
                                                    const double* __restrict__ v, const uint16_t* __restrict__ mask,
                                                    TZ* __restrict__ z, int bid) {
  const int n = bid * RB + threadIdx.x;
  if (n >= g.Npad) return;
  const unsigned m = (n < g.N) ? mask[n] : 0;
#pragma unroll
  for (int c = 0; c < NDOF; ++c) {
    const int64_t q = (int64_t)c * g.Npad + n;
    z[q] = ((m >> c) & 1) ? (TZ)v[q] : (TZ)x[q];
  }
}
template <typename T, typename TZ>
__global__ void __launch_bounds__(RB) precond_finish_kernel(Grid g, const T* __restrict__ x,
                                                            const double* __restrict__ v,
                                                            const uint16_t* __restrict__ mask, TZ* __restrict__ z) {
  precond_finish_body<T, TZ>(g, x, v, mask, z, blockIdx.x);
}

template <typename T, typename TZ>
void launch_precond_finish(const Grid& g, const T* x, const double* v, const uint16_t* mask, TZ* z, hipStream_t s) {
  precond_finish_kernel<T, TZ><<<(g.Npad + RB - 1) / RB, RB, 0, s>>>(g, x, v, mask, z);
}
template void launch_precond_finish<float, float>(const Grid&, const float*, const double*, const uint16_t*, float*,
                                                  hipStream_t);
template void launch_precond_finish<float, double>(const Grid&, const float*, const double*, const uint16_t*,
                                                   double*, hipStream_t);
template void launch_precond_finish<double, double>(const Grid&, const double*, const double*, const uint16_t*,
                                                    double*, hipStream_t);

// batched ends of the preconditioner: BOP_CONVERT b (y, T) = masked v (b,
// FP64); BOP_FINISH z (y, TZ) = x (T), v on constrained dofs
template <typename T>
__global__ void __launch_bounds__(RB) convert_masked_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  convert_masked_body<double, T>(j.g, (const double*)j.b, j.mask, (T*)j.y, bid);
}
template <typename T, typename TZ>
__global__ void __launch_bounds__(RB) precond_finish_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  precond_finish_body<T, TZ>(j.g, (const T*)j.x, (const double*)j.b, j.mask, (TZ*)j.y, bid);
}
template <typename T, typename TZ>
void launch_vec_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s) {
  if (op == BOP_CONVERT)
    convert_masked_batch<T><<<blocks, RB, 0, s>>>(jobs, njobs);
  else if (op == BOP_FINISH)
    precond_finish_batch<T, TZ><<<blocks, RB, 0, s>>>(jobs, njobs);
}
template void launch_vec_batch<float, float>(int, const BJob*, int, int, hipStream_t);
template void launch_vec_batch<float, double>(int, const BJob*, int, int, hipStream_t);
template void launch_vec_batch<double, double>(int, const BJob*, int, int, hipStream_t);
int vec_job_blocks(const Grid& g) { return (g.Npad + RB - 1) / RB; }

// ---- batched Krylov operations ---------------------------------------------------
__global__ void __launch_bounds__(RB) krylov_batch_kernel(int op, const KJob* __restrict__ jobs, int njobs) {
  int bid;
  const KJob& j = find_job(jobs, njobs, bid);
  switch (op) {  // uniform: one op per launch
    case KOP_MULTIDOT: multidot_body(j.n, j.V, j.n, j.k, j.w, j.part, bid, j.nblk); break;
    case KOP_REDUCE: reduce_body(j.nb, j.part, j.out, j.flag, bid); break;
    case KOP_MULTIAXPY: multiaxpy_body(j.n, j.V, j.n, j.k, j.h, j.w, j.flag ? j.part : nullptr, bid, j.nblk); break;
    case KOP_SCALE:
      for (int64_t i = (int64_t)bid * RB + threadIdx.x; i < j.n; i += (int64_t)j.nblk * RB)
        j.w[i] = j.a * j.w[i] + 0.0;  // as axpby with y = null
      break;
    case KOP_COPY:
      for (int i = threadIdx.x; i < j.k; i += RB) j.out[i] = j.src[i];
      break;
    default: break;
  }
}

int krylov_job_blocks(int op, const KJob& j) {
  switch (op) {
    case KOP_MULTIDOT:
    case KOP_MULTIAXPY: return red_blocks(j.n);
    case KOP_REDUCE: return j.k;
    case KOP_SCALE: return (int)std::min<int64_t>(1024, (j.n + RB - 1) / RB);
    case KOP_COPY: return 1;
    default: return 0;
  }
}

void launch_krylov_batch(int op, const KJob* jobs, int njobs, int blocks, hipStream_t s) {
  if (njobs > 0 && blocks > 0) krylov_batch_kernel<<<blocks, RB, 0, s>>>(op, jobs, njobs);
}

}  // namespace mvpf
