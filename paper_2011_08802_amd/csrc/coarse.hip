// Coarsest-level direct solve (Sec. 3.4: the V-cycle bottoms out in a sparse
// LU factorisation).  The coarsest operator (at most 8192 unknowns) is
// gathered into a dense FP64 matrix and inverted once per Newton system by
// Gauss-Jordan elimination with partial pivoting; each V-cycle then applies
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
  for (int s = 0; s < NSTEN; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    if (i + dx < 0 || i + dx >= g.nnx || j + dy < 0 || j + dy >= g.nny || k + dz < 0 || k + dz >= g.nnz) continue;
    const int m = n + dx + g.nnx * (dy + g.nny * dz);
    const double* Ab = A + ((int64_t)(t * NSTEN + s) * NBLK) * TILE + l;
    for (int r = 0; r < 9; ++r)
      for (int c = 0; c < 9; ++c)
        D[((int64_t)r * g.N + n) * nd + (int64_t)c * g.N + m] = Ab[(r * 9 + c) * TILE];
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

// Augmented matrix M = [A | I], n x 2n, row-major.  Step j: pick the pivot
// row (largest |M(i,j)|, i >= j), swap it into row j, scale row j, record the
// elimination factors of column j.
__global__ void __launch_bounds__(1024) gj_pivot_kernel(int n, int j, double* __restrict__ M,
                                                        double* __restrict__ fac, int* status) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x;
  const int64_t w = 2 * (int64_t)n;
  double best = -1.0;
  int bi = j;
  for (int i = j + tid; i < n; i += blockDim.x) {
    const double v = fabs(M[(int64_t)i * w + j]);
    if (v > best) { best = v; bi = i; }
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) {
      const double o = sv[tid + off];
      const int oi = si[tid + off];
      if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) { sv[tid] = o; si[tid] = oi; }
    }
    __syncthreads();
  }
  const int p = si[0];
  const double pv = sv[0];
  if (!(pv > 0.0)) {
    if (tid == 0) atomicOr(status, 1);
    // leave the matrix untouched; host reports the singular pivot
    for (int i = tid; i < n; i += blockDim.x) fac[i] = 0.0;
    return;
  }
  if (p != j)
    for (int64_t c = tid; c < w; c += blockDim.x) {
      const double a = M[(int64_t)j * w + c];
      M[(int64_t)j * w + c] = M[(int64_t)p * w + c];
      M[(int64_t)p * w + c] = a;
    }
  __syncthreads();
  const double ip = 1.0 / M[(int64_t)j * w + j];
  __syncthreads();
  for (int64_t c = tid; c < w; c += blockDim.x) M[(int64_t)j * w + c] *= ip;
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) fac[i] = (i == j) ? 0.0 : M[(int64_t)i * w + j];
}

__global__ void __launch_bounds__(256) gj_eliminate_kernel(int n, int j, double* __restrict__ M,
                                                           const double* __restrict__ fac) {
  const int64_t w = 2 * (int64_t)n;
  const int i = blockIdx.y;
  if (i == j) return;
  const double f = fac[i];
  if (f == 0.0) return;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < w; c += (int64_t)gridDim.x * blockDim.x)
    M[(int64_t)i * w + c] -= f * M[(int64_t)j * w + c];
}

__global__ void __launch_bounds__(256) gj_init_kernel(int n, const double* __restrict__ a, double* __restrict__ M) {
  const int64_t w = 2 * (int64_t)n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * w;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / w, c = idx - i * w;
    M[idx] = (c < n) ? a[i * n + c] : ((c - n == i) ? 1.0 : 0.0);
  }
}

__global__ void __launch_bounds__(256) gj_extract_kernel(int n, const double* __restrict__ M, double* __restrict__ inv) {
  const int64_t w = 2 * (int64_t)n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, c = idx - i * n;
    inv[idx] = M[i * w + n + c];
  }
}

// a: n x n input (not modified); inv: n x n output; work: >= 2 n^2 + n doubles.
int dense_invert(int n, double* a, double* inv, double* work, int* status, hipStream_t s) {
  double* M = work;
  double* fac = work + 2 * (int64_t)n * n;
  gj_init_kernel<<<1024, 256, 0, s>>>(n, a, M);
  const int gx = (int)std::min<int64_t>((2 * (int64_t)n + 255) / 256, 16);
  for (int j = 0; j < n; ++j) {
    gj_pivot_kernel<<<1, 1024, 0, s>>>(n, j, M, fac, status);
    gj_eliminate_kernel<<<dim3(gx, n), 256, 0, s>>>(n, j, M, fac);
  }
  gj_extract_kernel<<<1024, 256, 0, s>>>(n, M, inv);
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
