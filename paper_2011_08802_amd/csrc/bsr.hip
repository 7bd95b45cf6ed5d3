// 9x9-block operator kernels on the structured 27-point stencil.
//
// One thread per node row.  The operator is stored as symmetric half stencil,
// tiled structure-of-arrays (64 rows per tile, see common.h), so each operator
// load of a row is a fully coalesced 64-lane access (256 B in FP32, 512 B in
// FP64); vectors are component-major, so the 9 values of each neighbour are
// coalesced loads as well.  These kernels are HBM-bandwidth bound: per row
// they move 14*81*sizeof(TA) bytes of operator plus ~10 vector values, and
// 2*13*9 accumulation values for the transposed lower half.
#include "common.h"

namespace mvpf {

template <typename T>
struct Acc;
template <>
struct Acc<float> { using type = float; };
template <>
struct Acc<double> { using type = double; };

// Launch shape of the row kernels.  nb = ceil(Npad / 256) logical blocks of
// 256 rows.  With G = gridDim.x workgroups (a multiple of 8), workgroup b
// (which the hardware places on XCD b % 8) handles logical blocks
// L = r*G + (b % 8)*(G/8) + b/8 for rounds r = 0, 1, ...: within a round each
// XCD walks a contiguous range of rows, and only G*256 rows are in flight, so
// the transposed lower-half reads of neighbouring rows hit L2 / the infinity
// cache.  G >= nb is the plain one-block-per-256-rows launch.
__host__ __device__ inline int row_blocks(const Grid& g) { return (g.Npad + 255) / 256; }
inline int row_grid(const Grid& g, int G) {
  const int nb_pad = (row_blocks(g) + 7) / 8 * 8;
  if (G <= 0 || G >= nb_pad) return nb_pad;
  return std::max(8, G / 8 * 8);
}

// ROW_LOOP_B: the same for workgroup bid of nblk (a job of a batched launch)
#define ROW_LOOP_B(g, bid, nblk)                                                   \
  const int nb_ = row_blocks(g);                                                  \
  const int per_ = (nblk) >> 3;                                                    \
  for (int L_ = ((bid) & 7) * per_ + ((bid) >> 3); L_ < nb_; L_ += (nblk))         \
    for (int n = L_ * 256 + threadIdx.x, once_ = 1; once_; once_ = 0)
#define ROW_LOOP(g) ROW_LOOP_B(g, (int)blockIdx.x, (int)gridDim.x)

// Symmetric product in two passes, so that every stored block is read from
// memory exactly once whatever the cache does:
//  pass 1 (row n): acc_n (-)= sum_u A_u(n) x(n + off_u) over the 14 stored
//    blocks, and for the 13 off-diagonal ones the transposed contribution
//    A_u(n)^T x(n) to row m = n + off_u is written to C[u-1][.][m] (each
//    (u, m) has exactly one writer; lanes write consecutive m);
//  pass 2 (row m): acc_m (-)= sum_u C[u-1][.][m] over the in-grid lower
//    neighbours, then the kernel's epilogue (defect, Jacobi update, product).
// C holds 13 * NDOF * Npad values of the accumulation type.
// Stored blocks u0 .. u1 - 1 of row n (see upper_pass).
template <bool SUB, typename TA, typename TX, typename TC>
__device__ __forceinline__ void upper_range(const Grid& g, const TA* __restrict__ A, const TX* __restrict__ x, int n,
                                            int u0, int u1, TC acc[NDOF], TC* __restrict__ C) {
  const int t = n >> 6, l = n & 63;
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  TC xn[NDOF];
#pragma unroll
  for (int c = 0; c < NDOF; ++c) xn[c] = (TC)x[(int64_t)c * g.Npad + n];
#pragma unroll 1
  for (int u = u0; u < u1; ++u) {
    const int s = 13 + u;
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    if (!((i + dx >= 0) && (i + dx < g.nnx) && (j + dy >= 0) && (j + dy < g.nny) && (k + dz < g.nnz))) continue;
    const int m = n + dx + g.nnx * (dy + g.nny * dz);
    TC xv[NDOF];
#pragma unroll
    for (int c = 0; c < NDOF; ++c) xv[c] = (TC)x[(int64_t)c * g.Npad + m];
    using VT = typename Vec16<TA>::type;
    constexpr int V = Lay<TA>::V;
    const VT* Ab = reinterpret_cast<const VT*>(A + ((int64_t)t * NUP + u) * Lay<TA>::SLICE) + l;
    TC ct[NDOF] = {};
    TC sum[NDOF] = {};
#pragma unroll
    for (int q = 0; q < Lay<TA>::NQ; ++q) {
      const VT vq = Ab[q * TILE];
      TA av[V];
      __builtin_memcpy(av, &vq, sizeof(VT));
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int e = q * V + v;
        if (e < NBLK) {
          const int r = e / NDOF, c = e % NDOF;
          const TC a = (TC)av[v];
          sum[r] += a * xv[c];
          ct[c] += a * xn[r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NDOF; ++r) {
      if (SUB) acc[r] -= sum[r]; else acc[r] += sum[r];
    }
    if (u > 0) {
      TC* Cu = C + (int64_t)(u - 1) * NDOF * g.Npad + m;
#pragma unroll
      for (int c = 0; c < NDOF; ++c) Cu[(int64_t)c * g.Npad] = ct[c];
    }
  }
}

// The 14 stored blocks are summed in two halves, u < USPLIT into acc and
// u >= USPLIT into a separate partial that is then added (or subtracted):
// the split kernels give each half its own wavefront, and every kernel
// family uses this same order, so results do not depend on the launch shape.
constexpr int USPLIT = 7;

template <bool SUB, typename TA, typename TX, typename TC>
__device__ __forceinline__ void upper_pass(const Grid& g, const TA* __restrict__ A, const TX* __restrict__ x, int n,
                                           TC acc[NDOF], TC* __restrict__ C) {
  upper_range<SUB>(g, A, x, n, 0, USPLIT, acc, C);
  TC p1[NDOF] = {};
  upper_range<false>(g, A, x, n, USPLIT, NUP, p1, C);
#pragma unroll
  for (int r = 0; r < NDOF; ++r) {
    if (SUB) acc[r] -= p1[r]; else acc[r] += p1[r];
  }
}

template <bool SUB, typename TC>
__device__ __forceinline__ void lower_pass(const Grid& g, int m, TC acc[NDOF], const TC* __restrict__ C) {
  const int i = m % g.nnx, j = (m / g.nnx) % g.nny, k = m / (g.nnx * g.nny);
#pragma unroll
  for (int u = 1; u < NUP; ++u) {
    const int s = 13 + u;
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    if (!((i - dx >= 0) && (i - dx < g.nnx) && (j - dy >= 0) && (j - dy < g.nny) && (k - dz >= 0))) continue;
    const TC* Cu = C + (int64_t)(u - 1) * NDOF * g.Npad + m;
#pragma unroll
    for (int c = 0; c < NDOF; ++c) {
      if (SUB) acc[c] -= Cu[(int64_t)c * g.Npad]; else acc[c] += Cu[(int64_t)c * g.Npad];
    }
  }
}

// y = A x: pass 1 writes the upper part into y, pass 2 adds the lower part.
template <typename TA, typename TX, typename TY>
__global__ void __launch_bounds__(256) spmv_upper_kernel(Grid g, const TA* __restrict__ A, const TX* __restrict__ x,
                                                         TY* __restrict__ y, TY* __restrict__ C) {
  ROW_LOOP(g) {
    if (n >= g.Npad) continue;
    TY acc[NDOF] = {};
    if (n < g.N) upper_pass<false>(g, A, x, n, acc, C);
#pragma unroll
    for (int r = 0; r < NDOF; ++r) y[(int64_t)r * g.Npad + n] = acc[r];
  }
}

template <typename TY>
__global__ void __launch_bounds__(256) spmv_lower_kernel(Grid g, TY* __restrict__ y, const TY* __restrict__ C) {
  ROW_LOOP(g) {
    if (n >= g.N) continue;
    TY acc[NDOF];
#pragma unroll
    for (int r = 0; r < NDOF; ++r) acc[r] = y[(int64_t)r * g.Npad + n];
    lower_pass<false>(g, n, acc, C);
#pragma unroll
    for (int r = 0; r < NDOF; ++r) y[(int64_t)r * g.Npad + n] = acc[r];
  }
}

// Pass 1 with the two halves of each tile's blocks on two wavefronts: a
// workgroup = 2 tiles x 2 halves; the second half's partial row sums go
// through LDS to the first, which finishes the row (same order as
// upper_pass).  Twice as many, shorter wavefronts as the one-wave kernels.
__device__ __forceinline__ int split_tile(int b, int nb_pad) {
  const int per = nb_pad >> 3;
  return ((b & 7) * per + (b >> 3)) * 2;  // first tile of logical block (XCD-contiguous)
}
inline int split_grid(const Grid& g) { return ((g.ntiles + 1) / 2 + 7) / 8 * 8; }

template <typename TA, typename TX, typename TY>
__global__ void __launch_bounds__(256) spmv_upper_split_kernel(Grid g, const TA* __restrict__ A,
                                                               const TX* __restrict__ x, TY* __restrict__ y,
                                                               TY* __restrict__ C) {
  __shared__ TY sh[2][NDOF][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, tl = w >> 1, half = w & 1;
  const int t = split_tile(blockIdx.x, gridDim.x) + tl;
  const int n = t * TILE + l;
  const bool valid = t < g.ntiles;
  TY acc[NDOF] = {};
  if (valid && n < g.N) upper_range<false>(g, A, x, n, half ? USPLIT : 0, half ? NUP : USPLIT, acc, C);
  if (half) {
#pragma unroll
    for (int r = 0; r < NDOF; ++r) sh[tl][r][l] = acc[r];
  }
  __syncthreads();
  if (!half && valid) {
#pragma unroll
    for (int r = 0; r < NDOF; ++r) y[(int64_t)r * g.Npad + n] = acc[r] + sh[tl][r][l];
  }
}

template <typename TA, typename TX, typename TY>
void launch_spmv(const Grid& g, const TA* A, const TX* x, TY* y, void* C, hipStream_t s, int G) {
  const int nb = row_grid(g, G);
  // FP64 operators keep one wavefront per tile (2 waves per SIMD fit either
  // way and the split measured slower); FP32 ones split
  if (G <= 0 && sizeof(TA) == 4)
    spmv_upper_split_kernel<TA, TX, TY><<<split_grid(g), 256, 0, s>>>(g, A, x, y, (TY*)C);
  else
    spmv_upper_kernel<TA, TX, TY><<<nb, 256, 0, s>>>(g, A, x, y, (TY*)C);
  spmv_lower_kernel<TY><<<nb, 256, 0, s>>>(g, y, (const TY*)C);
}
template void launch_spmv<double, double, double>(const Grid&, const double*, const double*, double*, void*,
                                                  hipStream_t, int);
template void launch_spmv<double, float, double>(const Grid&, const double*, const float*, double*, void*,
                                                 hipStream_t, int);
template void launch_spmv<float, float, float>(const Grid&, const float*, const float*, float*, void*, hipStream_t,
                                               int);

// r = b - A x
template <typename T>
__global__ void __launch_bounds__(256) defect_upper_kernel(Grid g, const T* __restrict__ A, const T* __restrict__ x,
                                                           const T* __restrict__ b, T* __restrict__ r,
                                                           T* __restrict__ C) {
  ROW_LOOP(g) {
    if (n >= g.Npad) continue;
    T acc[NDOF];
#pragma unroll
    for (int c = 0; c < NDOF; ++c) acc[c] = b[(int64_t)c * g.Npad + n];
    if (n < g.N) upper_pass<true>(g, A, x, n, acc, C);
#pragma unroll
    for (int c = 0; c < NDOF; ++c) r[(int64_t)c * g.Npad + n] = (n < g.N) ? acc[c] : (T)0;
  }
}

template <typename T>
__device__ __forceinline__ void defect_lower_body(const Grid& g, T* __restrict__ r, const T* __restrict__ C, int bid,
                                                  int nblk) {
  ROW_LOOP_B(g, bid, nblk) {
    if (n >= g.N) continue;
    T acc[NDOF];
#pragma unroll
    for (int c = 0; c < NDOF; ++c) acc[c] = r[(int64_t)c * g.Npad + n];
    lower_pass<true>(g, n, acc, C);
#pragma unroll
    for (int c = 0; c < NDOF; ++c) r[(int64_t)c * g.Npad + n] = acc[c];
  }
}
template <typename T>
__global__ void __launch_bounds__(256) defect_lower_kernel(Grid g, T* __restrict__ r, const T* __restrict__ C) {
  defect_lower_body<T>(g, r, C, blockIdx.x, gridDim.x);
}

template <typename T>
__device__ __forceinline__ void defect_upper_split_body(const Grid& g, const T* __restrict__ A,
                                                        const T* __restrict__ x, const T* __restrict__ b,
                                                        T* __restrict__ r, T* __restrict__ C, int bid, int nblk) {
  __shared__ T sh[2][NDOF][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, tl = w >> 1, half = w & 1;
  const int t = split_tile(bid, nblk) + tl;
  const int n = t * TILE + l;
  const bool valid = t < g.ntiles;
  T acc[NDOF] = {};
  if (valid && !half) {
#pragma unroll
    for (int c = 0; c < NDOF; ++c) acc[c] = b[(int64_t)c * g.Npad + n];
  }
  if (valid && n < g.N) {
    if (half)
      upper_range<false>(g, A, x, n, USPLIT, NUP, acc, C);
    else
      upper_range<true>(g, A, x, n, 0, USPLIT, acc, C);
  }
  if (half) {
#pragma unroll
    for (int c = 0; c < NDOF; ++c) sh[tl][c][l] = acc[c];
  }
  __syncthreads();
  if (!half && valid) {
#pragma unroll
    for (int c = 0; c < NDOF; ++c) r[(int64_t)c * g.Npad + n] = (n < g.N) ? acc[c] - sh[tl][c][l] : (T)0;
  }
}
template <typename T>
__global__ void __launch_bounds__(256) defect_upper_split_kernel(Grid g, const T* __restrict__ A,
                                                                 const T* __restrict__ x, const T* __restrict__ b,
                                                                 T* __restrict__ r, T* __restrict__ C) {
  defect_upper_split_body<T>(g, A, x, b, r, C, blockIdx.x, gridDim.x);
}

template <typename T>
void launch_defect(const Grid& g, const T* A, const T* x, const T* b, T* r, void* C, hipStream_t s, int G) {
  const int nb = row_grid(g, G);
  if (G <= 0)
    defect_upper_split_kernel<T><<<split_grid(g), 256, 0, s>>>(g, A, x, b, r, (T*)C);
  else
    defect_upper_kernel<T><<<nb, 256, 0, s>>>(g, A, x, b, r, (T*)C);
  defect_lower_kernel<T><<<nb, 256, 0, s>>>(g, r, (const T*)C);
}
template void launch_defect<float>(const Grid&, const float*, const float*, const float*, float*, void*, hipStream_t,
                                   int);
template void launch_defect<double>(const Grid&, const double*, const double*, const double*, double*, void*,
                                    hipStream_t, int);

// Damped point-block Jacobi sweep (Sec. 3.4): xo = x + omega D^-1 (b - A x).
// Pass 1 leaves the partial residual in xo; pass 2 completes it and updates.
// With a zero initial guess the product with A vanishes: xo = omega D^-1 b.
template <typename T>
__device__ __forceinline__ void pbj_zero_body(const Grid& g, const T* __restrict__ Dinv, const T* __restrict__ b,
                                              T* __restrict__ xo, T omega, int bid, int nblk) {
  ROW_LOOP_B(g, bid, nblk) {
    if (n >= g.Npad) continue;
    const int t = n >> 6, l = n & 63;
    const T* Db = Dinv + (int64_t)t * Lay<T>::SLICE;
    T bv[NDOF];
#pragma unroll
    for (int c = 0; c < NDOF; ++c) bv[c] = b[(int64_t)c * g.Npad + n];
#pragma unroll
    for (int r = 0; r < NDOF; ++r) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < NDOF; ++c) s += Db[Lay<T>::off(r * NDOF + c, l)] * bv[c];
      xo[(int64_t)r * g.Npad + n] = (n < g.N) ? omega * s : (T)0;
    }
  }
}
template <typename T>
__global__ void __launch_bounds__(256) pbj_zero_kernel(Grid g, const T* __restrict__ Dinv, const T* __restrict__ b,
                                                       T* __restrict__ xo, T omega) {
  pbj_zero_body<T>(g, Dinv, b, xo, omega, blockIdx.x, gridDim.x);
}

template <typename T>
__device__ __forceinline__ void pbj_lower_body(const Grid& g, const T* __restrict__ Dinv, const T* __restrict__ x,
                                               T* __restrict__ xo, const T* __restrict__ C, T omega, int bid,
                                               int nblk) {
  ROW_LOOP_B(g, bid, nblk) {
    if (n >= g.N) continue;
    T res[NDOF];
#pragma unroll
    for (int c = 0; c < NDOF; ++c) res[c] = xo[(int64_t)c * g.Npad + n];
    lower_pass<true>(g, n, res, C);
    const int t = n >> 6, l = n & 63;
    const T* Db = Dinv + (int64_t)t * Lay<T>::SLICE;
#pragma unroll
    for (int r = 0; r < NDOF; ++r) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < NDOF; ++c) s += Db[Lay<T>::off(r * NDOF + c, l)] * res[c];
      xo[(int64_t)r * g.Npad + n] = x[(int64_t)r * g.Npad + n] + omega * s;
    }
  }
}
template <typename T>
__global__ void __launch_bounds__(256) pbj_lower_kernel(Grid g, const T* __restrict__ Dinv, const T* __restrict__ x,
                                                        T* __restrict__ xo, const T* __restrict__ C, T omega) {
  pbj_lower_body<T>(g, Dinv, x, xo, C, omega, blockIdx.x, gridDim.x);
}

template <typename T>
void launch_pbj(const Grid& g, const T* A, const T* Dinv, const T* x, const T* b, T* xo, T omega, bool zero_guess,
                void* C, hipStream_t s, int G) {
  const int nb = row_grid(g, G);
  if (zero_guess) {
    pbj_zero_kernel<T><<<nb, 256, 0, s>>>(g, Dinv, b, xo, omega);
    return;
  }
  if (G <= 0)
    defect_upper_split_kernel<T><<<split_grid(g), 256, 0, s>>>(g, A, x, b, xo, (T*)C);
  else
    defect_upper_kernel<T><<<nb, 256, 0, s>>>(g, A, x, b, xo, (T*)C);
  pbj_lower_kernel<T><<<nb, 256, 0, s>>>(g, Dinv, x, xo, (const T*)C, omega);
}
template void launch_pbj<float>(const Grid&, const float*, const float*, const float*, const float*, float*, float,
                                bool, void*, hipStream_t, int);
template void launch_pbj<double>(const Grid&, const double*, const double*, const double*, const double*, double*,
                                 double, bool, void*, hipStream_t, int);

// ---- small grids --------------------------------------------------------------
// On coarse levels the one-thread-per-row kernels are latency bound (27 rounds
// of dependent loads per thread).  Here 27 threads share a row, one per
// stencil block; each does one round of loads and the 27 partial products are
// summed through LDS in a fixed order.  9 rows per 256-thread workgroup,
// thread index = s * 9 + local row.
constexpr int SMALL_ROWS = 9;

template <typename T, bool PBJ>
__device__ __forceinline__ void row_small_body(const Grid& g, const T* __restrict__ A, const T* __restrict__ Dinv,
                                               const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ out,
                                               T omega, int bid) {
  __shared__ T part[SMALL_ROWS][NSTEN][NDOF];
  __shared__ T res[SMALL_ROWS][NDOF];
  const int tid = threadIdx.x;
  const int s = tid / SMALL_ROWS, ln = tid % SMALL_ROWS;
  const int n = bid * SMALL_ROWS + ln;
  T pr[NDOF] = {};
  if (tid < SMALL_ROWS * NSTEN && n < g.N) {
    const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    if (i + dx >= 0 && i + dx < g.nnx && j + dy >= 0 && j + dy < g.nny && k + dz >= 0 && k + dz < g.nnz) {
      const int m = n + dx + g.nnx * (dy + g.nny * dz);
      T xv[NDOF];
#pragma unroll
      for (int c = 0; c < NDOF; ++c) xv[c] = x[(int64_t)c * g.Npad + m];
      if (s >= 13) {
        const T* Ab = A + ((int64_t)(n >> 6) * NUP + (s - 13)) * Lay<T>::SLICE;
        const int ll = n & 63;
#pragma unroll
        for (int r = 0; r < NDOF; ++r) {
          T acc = 0;
#pragma unroll
          for (int c = 0; c < NDOF; ++c) acc += Ab[Lay<T>::off(r * NDOF + c, ll)] * xv[c];
          pr[r] = acc;
        }
      } else {
        const T* Ab = A + ((int64_t)(m >> 6) * NUP + (13 - s)) * Lay<T>::SLICE;
        const int ll = m & 63;
#pragma unroll
        for (int r = 0; r < NDOF; ++r) {
          T acc = 0;
#pragma unroll
          for (int c = 0; c < NDOF; ++c) acc += Ab[Lay<T>::off(c * NDOF + r, ll)] * xv[c];
          pr[r] = acc;
        }
      }
    }
  }
  if (tid < SMALL_ROWS * NSTEN)
#pragma unroll
    for (int r = 0; r < NDOF; ++r) part[ln][s][r] = pr[r];
  __syncthreads();
  const int ln2 = tid / NDOF, r2 = tid % NDOF;
  const int n2 = bid * SMALL_ROWS + ln2;
  const bool own = tid < SMALL_ROWS * NDOF && n2 < g.N;
  if (own) {
    T acc = b[(int64_t)r2 * g.Npad + n2];
    for (int ss = 0; ss < NSTEN; ++ss) acc -= part[ln2][ss][r2];
    res[ln2][r2] = acc;
  }
  __syncthreads();
  if (own) {
    if (!PBJ) {
      out[(int64_t)r2 * g.Npad + n2] = res[ln2][r2];
    } else {
      const T* Db = Dinv + (int64_t)(n2 >> 6) * Lay<T>::SLICE;
      T acc = 0;
#pragma unroll
      for (int c = 0; c < NDOF; ++c) acc += Db[Lay<T>::off(r2 * NDOF + c, n2 & 63)] * res[ln2][c];
      out[(int64_t)r2 * g.Npad + n2] = x[(int64_t)r2 * g.Npad + n2] + omega * acc;
    }
  }
}
template <typename T, bool PBJ>
__global__ void __launch_bounds__(256) row_small_kernel(Grid g, const T* __restrict__ A, const T* __restrict__ Dinv,
                                                        const T* __restrict__ x, const T* __restrict__ b,
                                                        T* __restrict__ out, T omega) {
  row_small_body<T, PBJ>(g, A, Dinv, x, b, out, omega, blockIdx.x);
}

template <typename T>
void launch_row_small(const Grid& g, const T* A, const T* Dinv, const T* x, const T* b, T* out, T omega, bool pbj,
                      hipStream_t s) {
  const int nb = (g.N + SMALL_ROWS - 1) / SMALL_ROWS;
  if (pbj)
    row_small_kernel<T, true><<<nb, 256, 0, s>>>(g, A, Dinv, x, b, out, omega);
  else
    row_small_kernel<T, false><<<nb, 256, 0, s>>>(g, A, Dinv, x, b, out, omega);
}
template void launch_row_small<float>(const Grid&, const float*, const float*, const float*, const float*, float*,
                                      float, bool, hipStream_t);
template void launch_row_small<double>(const Grid&, const double*, const double*, const double*, const double*,
                                       double*, double, bool, hipStream_t);

// ---- batched launches (one launch for the jobs of many problems) ------------
template <typename T>
__global__ void __launch_bounds__(256) pbj_zero_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  pbj_zero_body<T>(j.g, (const T*)j.D, (const T*)j.b, (T*)j.y, (T)j.omega, bid, j.nblk);
}
template <typename T>
__global__ void __launch_bounds__(256) defect_upper_split_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  defect_upper_split_body<T>(j.g, (const T*)j.A, (const T*)j.x, (const T*)j.b, (T*)j.y, (T*)j.C, bid, j.nblk);
}
template <typename T>
__global__ void __launch_bounds__(256) pbj_lower_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  pbj_lower_body<T>(j.g, (const T*)j.D, (const T*)j.x, (T*)j.y, (const T*)j.C, (T)j.omega, bid, j.nblk);
}
template <typename T>
__global__ void __launch_bounds__(256) defect_lower_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  defect_lower_body<T>(j.g, (T*)j.y, (const T*)j.C, bid, j.nblk);
}
template <typename T, bool PBJ>
__global__ void __launch_bounds__(256) row_small_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  row_small_body<T, PBJ>(j.g, (const T*)j.A, (const T*)j.D, (const T*)j.x, (const T*)j.b, (T*)j.y, (T)j.omega, bid);
}

template <typename T>
void launch_bsr_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s) {
  switch (op) {
    case BOP_PBJ_ZERO: pbj_zero_batch<T><<<blocks, 256, 0, s>>>(jobs, njobs); break;
    case BOP_DEFECT_SPLIT: defect_upper_split_batch<T><<<blocks, 256, 0, s>>>(jobs, njobs); break;
    case BOP_PBJ_LOWER: pbj_lower_batch<T><<<blocks, 256, 0, s>>>(jobs, njobs); break;
    case BOP_DEFECT_LOWER: defect_lower_batch<T><<<blocks, 256, 0, s>>>(jobs, njobs); break;
    case BOP_ROW_SMALL_PBJ: row_small_batch<T, true><<<blocks, 256, 0, s>>>(jobs, njobs); break;
    case BOP_ROW_SMALL_DEFECT: row_small_batch<T, false><<<blocks, 256, 0, s>>>(jobs, njobs); break;
    default: break;
  }
}
template void launch_bsr_batch<float>(int, const BJob*, int, int, hipStream_t);
template void launch_bsr_batch<double>(int, const BJob*, int, int, hipStream_t);

// workgroups of one job (plain shapes: one logical block of 256 rows per
// workgroup, rounded up to whole rounds over the 8 XCDs)
int bsr_job_blocks(int op, const Grid& g) {
  switch (op) {
    case BOP_PBJ_ZERO:
    case BOP_PBJ_LOWER:
    case BOP_DEFECT_LOWER: return row_grid(g, 0);
    case BOP_DEFECT_SPLIT: return split_grid(g);
    case BOP_ROW_SMALL_PBJ:
    case BOP_ROW_SMALL_DEFECT: return (g.N + SMALL_ROWS - 1) / SMALL_ROWS;
    default: return 0;
  }
}

}  // namespace mvpf
