// 9x9-block operator kernels on the structured 27-point stencil.
//
// One thread per node row.  The operator is stored tiled structure-of-arrays
// (64 rows per tile, see common.h), so each of the 27*81 loads of a row is a
// fully coalesced 64-lane access (256 B in FP32, 512 B in FP64); the vector
// is stored component-major, so the 9 neighbour values of each stencil point
// are also coalesced 64-lane loads and largely L1/L2 hits (neighbouring rows
// share them).  These kernels are HBM-bandwidth bound: per row they move
// 27*81*sizeof(TA) bytes of operator plus ~10 vector values.
#include "common.h"

namespace mvpf {

template <typename T>
struct Acc;
template <>
struct Acc<float> { using type = float; };
template <>
struct Acc<double> { using type = double; };

// acc[r] -= sum_s sum_c A(n, s)[r][c] * x[c][n + off(s)]   (SUB) or +=
template <bool SUB, typename TA, typename TX, typename TC>
__device__ __forceinline__ void row_product(const Grid& g, const TA* __restrict__ A, const TX* __restrict__ x,
                                            int n, TC acc[9]) {
  const int t = n >> 6, l = n & 63;
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  const TA* Arow = A + (int64_t)t * NSTEN * NBLK * TILE + l;
#pragma unroll 1
  for (int s = 0; s < NSTEN; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    const bool valid = (i + dx >= 0) && (i + dx < g.nnx) && (j + dy >= 0) && (j + dy < g.nny) &&
                       (k + dz >= 0) && (k + dz < g.nnz);
    if (!valid) continue;
    const int m = n + dx + g.nnx * (dy + g.nny * dz);
    TC xv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) xv[c] = (TC)x[(int64_t)c * g.Npad + m];
    const TA* Ab = Arow + (int64_t)s * NBLK * TILE;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      TC sum = 0;
#pragma unroll
      for (int c = 0; c < 9; ++c) sum += (TC)Ab[(r * 9 + c) * TILE] * xv[c];
      if (SUB)
        acc[r] -= sum;
      else
        acc[r] += sum;
    }
  }
}

template <typename TA, typename TX, typename TY>
__global__ void __launch_bounds__(256) spmv_kernel(Grid g, const TA* __restrict__ A, const TX* __restrict__ x,
                                                   TY* __restrict__ y) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.Npad) return;
  using TC = typename Acc<TY>::type;
  TC acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (n < g.N) row_product<false>(g, A, x, n, acc);
#pragma unroll
  for (int r = 0; r < 9; ++r) y[(int64_t)r * g.Npad + n] = (TY)acc[r];
}

template <typename TA, typename TX, typename TY>
void launch_spmv(const Grid& g, const TA* A, const TX* x, TY* y, hipStream_t s) {
  spmv_kernel<TA, TX, TY><<<(g.Npad + 255) / 256, 256, 0, s>>>(g, A, x, y);
}
template void launch_spmv<double, double, double>(const Grid&, const double*, const double*, double*, hipStream_t);
template void launch_spmv<double, float, double>(const Grid&, const double*, const float*, double*, hipStream_t);
template void launch_spmv<float, float, float>(const Grid&, const float*, const float*, float*, hipStream_t);

// r = b - A x
template <typename T>
__global__ void __launch_bounds__(256) defect_kernel(Grid g, const T* __restrict__ A, const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ r) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.Npad) return;
  T acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = b[(int64_t)c * g.Npad + n];
  if (n < g.N) row_product<true>(g, A, x, n, acc);
#pragma unroll
  for (int c = 0; c < 9; ++c) r[(int64_t)c * g.Npad + n] = (n < g.N) ? acc[c] : (T)0;
}

template <typename T>
void launch_defect(const Grid& g, const T* A, const T* x, const T* b, T* r, hipStream_t s) {
  defect_kernel<T><<<(g.Npad + 255) / 256, 256, 0, s>>>(g, A, x, b, r);
}
template void launch_defect<float>(const Grid&, const float*, const float*, const float*, float*, hipStream_t);
template void launch_defect<double>(const Grid&, const double*, const double*, const double*, double*, hipStream_t);

// Damped point-block Jacobi sweep (Sec. 3.4): xo = x + omega D^-1 (b - A x);
// with a zero initial guess the product with A vanishes: xo = omega D^-1 b.
template <typename T, bool ZERO>
__global__ void __launch_bounds__(256) pbj_kernel(Grid g, const T* __restrict__ A, const T* __restrict__ Dinv,
                                                  const T* __restrict__ x, const T* __restrict__ b,
                                                  T* __restrict__ xo, T omega) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.Npad) return;
  if (n >= g.N) {
#pragma unroll
    for (int c = 0; c < 9; ++c) xo[(int64_t)c * g.Npad + n] = (T)0;
    return;
  }
  T res[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) res[c] = b[(int64_t)c * g.Npad + n];
  if (!ZERO) row_product<true>(g, A, x, n, res);
  const int t = n >> 6, l = n & 63;
  const T* Db = Dinv + (int64_t)t * NBLK * TILE + l;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    T s = 0;
#pragma unroll
    for (int c = 0; c < 9; ++c) s += Db[(r * 9 + c) * TILE] * res[c];
    const T x0 = ZERO ? (T)0 : x[(int64_t)r * g.Npad + n];
    xo[(int64_t)r * g.Npad + n] = x0 + omega * s;
  }
}

template <typename T>
void launch_pbj(const Grid& g, const T* A, const T* Dinv, const T* x, const T* b, T* xo, T omega,
                bool zero_guess, hipStream_t s) {
  const int nb = (g.Npad + 255) / 256;
  if (zero_guess)
    pbj_kernel<T, true><<<nb, 256, 0, s>>>(g, A, Dinv, x, b, xo, omega);
  else
    pbj_kernel<T, false><<<nb, 256, 0, s>>>(g, A, Dinv, x, b, xo, omega);
}
template void launch_pbj<float>(const Grid&, const float*, const float*, const float*, const float*, float*, float,
                                bool, hipStream_t);
template void launch_pbj<double>(const Grid&, const double*, const double*, const double*, const double*, double*,
                                 double, bool, hipStream_t);

}  // namespace mvpf
