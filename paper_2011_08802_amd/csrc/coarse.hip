// Coarsest-level direct solve (Sec. 3.4: the V-cycle bottoms out in a sparse
// LU factorisation).  The coarsest operator (at most 8192 unknowns) is
// gathered into a dense FP64 matrix and inverted once per Newton system by
// blocked Gauss-Jordan elimination with partial pivoting; each V-cycle then applies
// the inverse with one dense matrix-vector product (fully parallel, instead
// of two latency-bound triangular solves).
//
// Dense unknown ordering: d = c * N + n (component-major, no padding).
#include "common.h"

namespace mvpf {

__global__ void __launch_bounds__(256) dense_from_bsr_kernel(Grid g, const double* __restrict__ A,
                                                             double* __restrict__ D) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int64_t nd = (int64_t)NDOF * g.N;
  const int t = n >> 6, l = n & 63;
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  for (int u = 0; u < NUP; ++u) {
    const int s = 13 + u;
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    if (i + dx < 0 || i + dx >= g.nnx || j + dy < 0 || j + dy >= g.nny || k + dz < 0 || k + dz >= g.nnz) continue;
    const int m = n + dx + g.nnx * (dy + g.nny * dz);
    const double* Ab = A + (int64_t)(t * NUP + u) * Lay<double>::SLICE;
    for (int r = 0; r < 9; ++r)
      for (int c = 0; c < 9; ++c) {
        const double v = Ab[Lay<double>::off(r * 9 + c, l)];
        D[((int64_t)r * g.N + n) * nd + (int64_t)c * g.N + m] = v;
        if (u > 0) D[((int64_t)c * g.N + m) * nd + (int64_t)r * g.N + n] = v;  // lower half by symmetry
      }
  }
}

__global__ void zero_kernel_d(int64_t n, double* p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

void launch_dense_from_bsr(const Grid& g, const double* A64, double* dense, hipStream_t s) {
  const int64_t nd = (int64_t)NDOF * g.N;
  zero_kernel_d<<<1024, 256, 0, s>>>(nd * nd, dense);
  dense_from_bsr_kernel<<<(g.N + 255) / 256, 256, 0, s>>>(g, A64, dense);
}

// Blocked Gauss-Jordan inversion with partial pivoting on the augmented
// matrix M = [A | I] (n x 2n, row-major), panels of GJB columns.  For panel
// columns c0..c0+B-1:
//   1. gj_panel: one workgroup snapshots the panel F = M[:, panel] (kept in
//      registers), chooses the pivot rows P by Gauss-Jordan with partial
//      pivoting restricted to the panel (rows pivoted earlier are excluded),
//      and inverts the B x B pivot block Mp = F[P, :] (Gauss-Jordan with
//      partial pivoting in LDS);
//   2. gj_rows: R = Mp^-1 M[P, :] (the new pivot rows);
//   3. gj_update: rows in P become R, every other row i becomes
//      M[i, :] - F[i, :] R, which zeroes its panel columns.
// After the last panel the left half is a permutation (row prow[c] holds the
// unit entry of column c) and A^-1 row c = right half of row prow[c].
constexpr int GJB = 32;
constexpr int GJ_THREADS = 512;

// argmax of v (ties: lowest index; idx < 0 = no candidate) over the block
__device__ __forceinline__ void block_argmax(double& v, int& idx, double* sv, int* si) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off, 64);
    const int oi = __shfl_down(idx, off, 64);
    if (oi >= 0 && (ov > v || (ov == v && (idx < 0 || oi < idx)))) { v = ov; idx = oi; }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { sv[wid] = v; si[wid] = idx; }
  __syncthreads();
  if (wid == 0) {
    v = (lane < (int)(blockDim.x >> 6)) ? sv[lane] : -1.0;
    idx = (lane < (int)(blockDim.x >> 6)) ? si[lane] : -1;
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_down(v, off, 64);
      const int oi = __shfl_down(idx, off, 64);
      if (oi >= 0 && (ov > v || (ov == v && (idx < 0 || oi < idx)))) { v = ov; idx = oi; }
    }
    if (lane == 0) { sv[0] = v; si[0] = idx; }
  }
  __syncthreads();
  v = sv[0];
  idx = si[0];
}

// Panel factorisation.  Thread t owns rows t, t + GJ_THREADS, ... (RPT of
// them) and keeps their panel entries (PB <= GJB columns) in registers; the
// pivot row is broadcast through LDS.  n <= GJ_THREADS * RPT, B <= PB.
template <int RPT, int PB>
__global__ void __launch_bounds__(GJ_THREADS) gj_panel_kernel(int n, int c0, int B, const double* __restrict__ M,
                                                              double* __restrict__ F, int* __restrict__ done,
                                                              int* __restrict__ prow, int* __restrict__ pos,
                                                              double* __restrict__ Pinv, int* status) {
  __shared__ double sv[GJ_THREADS / 64];
  __shared__ int si[GJ_THREADS / 64];
  __shared__ double prowv[PB];
  __shared__ double Mp[PB][2 * PB];
  __shared__ double fr[PB];
  __shared__ int pr[PB];
  const int tid = threadIdx.x;
  const int64_t w = 2 * (int64_t)n;
  double W[RPT][PB];
  bool act[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = tid + q * GJ_THREADS;
    act[q] = i < n && !done[i];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      const double v = (i < n && b < B) ? M[(int64_t)i * w + c0 + b] : 0.0;
      W[q][b] = v;
      if (i < n && b < B) F[(int64_t)i * B + b] = v;
    }
  }
  // Register window: after each step the rows' entries shift left by one, so
  // the active panel column is always W[q][0] (all register indices static).
#pragma unroll 1
  for (int jj = 0; jj < B; ++jj) {
    double v = -1.0;
    int idx = -1;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const double cand = fabs(W[q][0]);
      if (act[q] && cand > v) { v = cand; idx = tid + q * GJ_THREADS; }
    }
    block_argmax(v, idx, sv, si);
    if (!(v > 0.0) || idx < 0) {
      if (tid == 0) atomicOr(status, 1);
      return;  // uniform
    }
    const int p = idx;
    if (p % GJ_THREADS == tid) {
      const int q = p / GJ_THREADS;
#pragma unroll
      for (int qq = 0; qq < RPT; ++qq)
        if (qq == q) {
          act[qq] = false;
#pragma unroll
          for (int b = 0; b < PB; ++b) prowv[b] = W[qq][b];
        }
      done[p] = 1;
      prow[c0 + jj] = p;
      pos[p] = c0 + jj;
      pr[jj] = p;
    }
    __syncthreads();
    const double ip = 1.0 / prowv[0];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const double f = act[q] ? W[q][0] * ip : 0.0;
#pragma unroll
      for (int b = 1; b < PB; ++b) W[q][b - 1] = W[q][b] - f * prowv[b];
      W[q][PB - 1] = 0.0;
    }
    __syncthreads();
  }
  // invert the pivot block Mp = F[P, :] (B x B) with partial pivoting, [Mp | I] in LDS
  for (int idx = tid; idx < B * B; idx += blockDim.x) {
    const int a = idx / B, b = idx % B;
    Mp[a][b] = F[(int64_t)pr[a] * B + b];
    Mp[a][B + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < B; ++c) {
    if (tid == 0) {
      int q = c;
      double bv = fabs(Mp[c][c]);
      for (int r = c + 1; r < B; ++r)
        if (fabs(Mp[r][c]) > bv) { bv = fabs(Mp[r][c]); q = r; }
      si[0] = q;
      sv[0] = bv;
    }
    __syncthreads();
    const int q = si[0];
    if (!(sv[0] > 0.0)) {
      if (tid == 0) atomicOr(status, 1);
      return;
    }
    if (q != c && tid < 2 * B) {
      const double tmp = Mp[c][tid];
      Mp[c][tid] = Mp[q][tid];
      Mp[q][tid] = tmp;
    }
    __syncthreads();
    const double ipc = 1.0 / Mp[c][c];
    __syncthreads();
    if (tid < 2 * B) Mp[c][tid] *= ipc;
    if (tid < B) fr[tid] = (tid == c) ? 0.0 : Mp[tid][c];
    __syncthreads();
    for (int idx = tid; idx < B * 2 * B; idx += blockDim.x) {
      const int r = idx / (2 * B), cc = idx % (2 * B);
      if (r != c) Mp[r][cc] -= fr[r] * Mp[c][cc];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < B * B; idx += blockDim.x) Pinv[idx] = Mp[idx / B][B + idx % B];
}

// R[a][c] = sum_b Pinv[a][b] M[prow[c0 + b]][c]
__global__ void __launch_bounds__(256) gj_rows_kernel(int n, int c0, int B, const double* __restrict__ M,
                                                      const int* __restrict__ prow, const double* __restrict__ Pinv,
                                                      double* __restrict__ R) {
  const int64_t w = 2 * (int64_t)n;
  const int a = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < w; c += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += Pinv[a * B + b] * M[(int64_t)prow[c0 + b] * w + c];
    R[(int64_t)a * w + c] = s;
  }
}

// M[i][c] = R[pos(i)][c] for pivot rows of this panel, else M[i][c] - F[i,:] R[:, c].
// Block: 32 rows x 256 columns; R column strip kept in registers.
__global__ void __launch_bounds__(256) gj_update_kernel(int n, int c0, int B, double* __restrict__ M,
                                                        const double* __restrict__ F, const double* __restrict__ R,
                                                        const int* __restrict__ pos) {
  __shared__ double Fs[32][GJB];
  const int64_t w = 2 * (int64_t)n;
  const int r0 = blockIdx.y * 32;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int idx = threadIdx.x; idx < 32 * GJB; idx += 256) {
    const int rr = idx / GJB, b = idx % GJB;
    Fs[rr][b] = (r0 + rr < n && b < B) ? F[(int64_t)(r0 + rr) * B + b] : 0.0;
  }
  __syncthreads();
  if (c >= w) return;
  double Rc[GJB];
#pragma unroll
  for (int b = 0; b < GJB; ++b) Rc[b] = (b < B) ? R[(int64_t)b * w + c] : 0.0;
  for (int rr = 0; rr < 32; ++rr) {
    const int i = r0 + rr;
    if (i >= n) break;
    const int pi = pos[i];
    double v;
    if (pi >= c0 && pi < c0 + B) {
      v = Rc[0];
#pragma unroll
      for (int b = 1; b < GJB; ++b)
        if (b == pi - c0) v = Rc[b];
    } else {
      v = M[(int64_t)i * w + c];
#pragma unroll
      for (int b = 0; b < GJB; ++b) v -= Fs[rr][b] * Rc[b];
    }
    M[(int64_t)i * w + c] = v;
  }
}

__global__ void __launch_bounds__(256) gj_init_kernel(int n, const double* __restrict__ a, double* __restrict__ M,
                                                      int* __restrict__ done, int* __restrict__ pos) {
  const int64_t w = 2 * (int64_t)n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * w;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / w, c = idx - i * w;
    M[idx] = (c < n) ? a[i * n + c] : ((c - n == i) ? 1.0 : 0.0);
    if (c == 0) { done[i] = 0; pos[i] = -1; }
  }
}

__global__ void __launch_bounds__(256) gj_extract_kernel(int n, const double* __restrict__ M,
                                                         const int* __restrict__ prow, double* __restrict__ inv) {
  const int64_t w = 2 * (int64_t)n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, c = idx - i * n;
    inv[idx] = M[(int64_t)prow[i] * w + n + c];
  }
}

size_t dense_invert_work(int n) {
  // M (2n^2) + F, W (n*GJB each) + R (GJB*2n) + Pinv (GJB^2) doubles, then 3n ints
  return (size_t)(2 * (int64_t)n * n + 2 * (int64_t)n * GJB + 2 * (int64_t)GJB * n + GJB * GJB) * sizeof(double) +
         (size_t)3 * n * sizeof(int);
}

// a: n x n input (not modified); inv: n x n output; work: dense_invert_work(n) bytes.
int dense_invert(int n, double* a, double* inv, double* work, int* status, hipStream_t s) {
  double* M = work;
  double* F = M + 2 * (int64_t)n * n;
  double* W = F + (int64_t)n * GJB;
  double* R = W + (int64_t)n * GJB;
  double* Pinv = R + 2 * (int64_t)GJB * n;
  int* done = (int*)(Pinv + GJB * GJB);
  int* prow = done + n;
  int* pos = prow + n;
  gj_init_kernel<<<1024, 256, 0, s>>>(n, a, M, done, pos);
  const int64_t w = 2 * (int64_t)n;
  // panel width: the rows' panel entries must fit in registers
  const int PBW = n <= 2 * GJ_THREADS ? 32 : n <= 4 * GJ_THREADS ? 16 : n <= 8 * GJ_THREADS ? 8 : 4;
  for (int c0 = 0; c0 < n; c0 += PBW) {
    const int B = std::min(PBW, n - c0);
    if (n <= GJ_THREADS)
      gj_panel_kernel<1, 32><<<1, GJ_THREADS, 0, s>>>(n, c0, B, M, F, done, prow, pos, Pinv, status);
    else if (n <= 2 * GJ_THREADS)
      gj_panel_kernel<2, 32><<<1, GJ_THREADS, 0, s>>>(n, c0, B, M, F, done, prow, pos, Pinv, status);
    else if (n <= 3 * GJ_THREADS)
      gj_panel_kernel<3, 16><<<1, GJ_THREADS, 0, s>>>(n, c0, B, M, F, done, prow, pos, Pinv, status);
    else if (n <= 4 * GJ_THREADS)
      gj_panel_kernel<4, 16><<<1, GJ_THREADS, 0, s>>>(n, c0, B, M, F, done, prow, pos, Pinv, status);
    else if (n <= 8 * GJ_THREADS)
      gj_panel_kernel<8, 8><<<1, GJ_THREADS, 0, s>>>(n, c0, B, M, F, done, prow, pos, Pinv, status);
    else
      gj_panel_kernel<16, 4><<<1, GJ_THREADS, 0, s>>>(n, c0, B, M, F, done, prow, pos, Pinv, status);
    gj_rows_kernel<<<dim3((int)std::min<int64_t>((w + 255) / 256, 64), B), 256, 0, s>>>(n, c0, B, M, prow, Pinv, R);
    gj_update_kernel<<<dim3((int)((w + 255) / 256), (n + 31) / 32), 256, 0, s>>>(n, c0, B, M, F, R, pos);
  }
  gj_extract_kernel<<<1024, 256, 0, s>>>(n, M, prow, inv);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// x = Ainv b on the coarsest level; one wavefront per output unknown, FP64
// accumulation; b and x are level vectors (component-major, padded).
template <typename T>
__global__ void __launch_bounds__(256) coarse_solve_kernel(Grid g, const double* __restrict__ Ainv,
                                                           const T* __restrict__ b, T* __restrict__ x) {
  const int64_t nd = (int64_t)NDOF * g.N;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nd) return;
  double s = 0.0;
  const double* Ar = Ainv + (int64_t)row * nd;
  for (int64_t c = lane; c < nd; c += 64) {
    const int comp = (int)(c / g.N), node = (int)(c - (int64_t)comp * g.N);
    s += Ar[c] * (double)b[(int64_t)comp * g.Npad + node];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) {
    const int comp = row / g.N, node = row - comp * g.N;
    x[(int64_t)comp * g.Npad + node] = (T)s;
  }
}

template <typename T>
void launch_coarse_solve(const Grid& g, const double* Ainv, const T* b, T* x, hipStream_t s) {
  const int64_t nd = (int64_t)NDOF * g.N;
  coarse_solve_kernel<T><<<(int)((nd + 3) / 4), 256, 0, s>>>(g, Ainv, b, x);
}
template void launch_coarse_solve<float>(const Grid&, const double*, const float*, float*, hipStream_t);
template void launch_coarse_solve<double>(const Grid&, const double*, const double*, double*, hipStream_t);

}  // namespace mvpf
