// Matrix-free application of the finest-level tangent from its Gauss-point
// Hessians (Sec. 3.4: K = d^2 Pi / dU^2, here never assembled on the finest
// level).  With v_g = B_g x_e the 15 local variables of Gauss point g
// (reference-cube gradients of u, h * eta) and D_g the packed 15 x 15 Hessian
// of the density,
//   (K x)_a = h/8 sum_g B_{g,a}^T D_g v_g  +  the gradient-energy term
//             h/8 sum_g dN_a . (Mg (x) I) grad_ref eta,
// which is the element matrix of the assembled path applied to x_e (same
// 2x2x2 rule; the Laplacian term is exact under it).
//
// Stored per element: 8 x 120 Hessian values (3.8 KB in FP32) instead of the
// half-stencil blocks of its node (4.7 KB) plus the assembled path's
// transposed contributions (0.9 KB written and read per sweep).
//
// Kernel layout: a wavefront covers 8 elements x 8 Gauss points (lane =
// 8 * element + point).  Each lane forms v_g, w = D_g v_g and the gradient
// energy's Mg grad eta, then its contributions to all 8 nodes of the element;
// a reduce-scatter over the 8 point lanes (xor 4, 2, 1) leaves lane g with
// the sum for node a = g, written to the element-output buffer.  A node
// gather sums its <= 8 elements in a fixed order and applies the epilogue
// (product, defect or damped point-block Jacobi update), so results are
// reproducible bit for bit.
#include "common.h"

namespace mvpf {

constexpr double MGQ0 = 0.21132486540518711775;  // (1 - 1/sqrt 3) / 2
constexpr double MGQ1 = 0.78867513459481288225;

// Contribution of one Gauss point to node a: c1 * B_a^T [w; z]
template <typename T>
__device__ __forceinline__ void node_part(int a, const T xg[3], const T w[15], const T z[18], T h, T c1, T out[9]) {
  T f[3], df[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool bit = (a >> d) & 1;
    f[d] = bit ? xg[d] : (T)1 - xg[d];
    df[d] = bit ? (T)1 : (T)-1;
  }
  const T N = f[0] * f[1] * f[2];
  const T dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i) out[i] = c1 * (dN[0] * w[3 * i] + dN[1] * w[3 * i + 1] + dN[2] * w[3 * i + 2]);
#pragma unroll
  for (int m = 0; m < 6; ++m)
    out[3 + m] = c1 * (h * N * w[9 + m] + dN[0] * z[3 * m] + dN[1] * z[3 * m + 1] + dN[2] * z[3 * m + 2]);
}

// E = element parts of K x_e (x masked on constrained dofs when mask != null).
// MINB: workgroups per CU the register budget is sized for (3 keeps the FP64
// product with FP32 input at 3 waves per SIMD without spills).
template <typename TD, typename TX, typename T, int MINB>
__global__ void __launch_bounds__(256, MINB) mf_element_kernel(Grid g, const TD* __restrict__ D, const TX* __restrict__ x,
                                                         const uint16_t* __restrict__ mask,
                                                         const DevCard* __restrict__ cd, T* __restrict__ E) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int gp = lane & 7;
  const int64_t e = (t >> 6) * 8 + (lane >> 3);
  const bool active = e < g.NE;  // inactive lanes still take part in the shuffles
  const T h = (T)g.h, c1 = (T)(0.125 * g.h);
  const T xg[3] = {(T)((gp & 1) ? MGQ1 : MGQ0), (T)((gp & 2) ? MGQ1 : MGQ0), (T)((gp & 4) ? MGQ1 : MGQ0)};
  T v[15], ge[18];
#pragma unroll
  for (int k = 0; k < 15; ++k) v[k] = 0;
#pragma unroll
  for (int k = 0; k < 18; ++k) ge[k] = 0;
  if (active) {
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int node = (ex + (a & 1)) + g.nnx * ((ey + ((a >> 1) & 1)) + g.nny * (ez + ((a >> 2) & 1)));
      const unsigned mb = mask ? mask[node] : 0u;
      T f[3], df[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const bool bit = (a >> d) & 1;
        f[d] = bit ? xg[d] : (T)1 - xg[d];
        df[d] = bit ? (T)1 : (T)-1;
      }
      const T N = f[0] * f[1] * f[2];
      const T dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const T xl = (T)x[(int64_t)c * g.Npad + node];  // unconditional load, then select
        const T xv = ((mb >> c) & 1) ? (T)0 : xl;
        if (c < 3) {
#pragma unroll
          for (int j = 0; j < 3; ++j) v[3 * c + j] += dN[j] * xv;
        } else {
          v[9 + c - 3] += h * N * xv;
#pragma unroll
          for (int j = 0; j < 3; ++j) ge[3 * (c - 3) + j] += dN[j] * xv;
        }
      }
    }
  }
  // w = D v (packed upper triangle, row-major p <= q), 16-byte loads; an
  // element whose unknowns are all zero (the lifting of a prescribed
  // increment touches few) contributes nothing and reads no Hessians
  bool nonzero = false;
#pragma unroll
  for (int k = 0; k < 15; ++k) nonzero = nonzero || v[k] != (T)0;
#pragma unroll
  for (int k = 0; k < 18; ++k) nonzero = nonzero || ge[k] != (T)0;
  T w[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) w[k] = 0;
  if (active && nonzero) {
    // streamed once per product: non-temporal 16-byte loads keep x and the
    // element outputs in the caches
    constexpr int V = 16 / (int)sizeof(TD);
    typedef TD VT __attribute__((ext_vector_type(V)));
    const VT* Dp = reinterpret_cast<const VT*>(D) + ((e >> 3) * 64 + gp * 8 + (e & 7));
    const int64_t ks = (int64_t)(g.NEpad >> 3) * 64;
    TD dv[V];
#pragma unroll
    for (int p = 0, k = 0; p < 15; ++p)
#pragma unroll
      for (int q = p; q < 15; ++q, ++k) {
        if (k % V == 0) {
          const VT vq = __builtin_nontemporal_load(Dp + (k / V) * ks);
          __builtin_memcpy(dv, &vq, sizeof(VT));
        }
        const T d = (T)dv[k % V];
        w[p] += d * v[q];
        if (q != p) w[q] += d * v[p];
      }
  }
  // gradient energy: z = (Mg (x) I) grad_ref eta
  T z[18];
#pragma unroll
  for (int m = 0; m < 6; ++m)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T s = 0;
#pragma unroll
      for (int m2 = 0; m2 < 6; ++m2) s += (T)cd->Mg[m][m2] * ge[3 * m2 + j];
      z[3 * m + j] = s;
    }
  // reduce-scatter over the 8 point lanes of the element
  const int b2 = (gp >> 2) & 1, b1 = (gp >> 1) & 1, b0 = gp & 1;
  T acc1[4][9];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T mine[9], other[9];
    node_part<T>(4 * b2 + k, xg, w, z, h, c1, mine);
    node_part<T>(4 * (1 - b2) + k, xg, w, z, h, c1, other);
#pragma unroll
    for (int c = 0; c < 9; ++c) acc1[k][c] = mine[c] + __shfl_xor(other[c], 4, 64);
  }
  T acc2[2][9];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const T mine = b1 ? acc1[2 + j][c] : acc1[j][c];
      const T other = b1 ? acc1[j][c] : acc1[2 + j][c];
      acc2[j][c] = mine + __shfl_xor(other, 2, 64);
    }
  T out[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const T mine = b0 ? acc2[1][c] : acc2[0][c];
    const T other = b0 ? acc2[0][c] : acc2[1][c];
    out[c] = mine + __shfl_xor(other, 1, 64);
  }
  if (active) {
#pragma unroll
    for (int c = 0; c < 9; ++c) E[eo_index(gp, c, e)] = out[c];
  }
}

// Node gather with epilogue.  MODE 0: y = K x; 1: r = b - K x;
// 2: xo = x + omega Dinv (b - K x).  Constrained rows (mask) act as the
// identity, as in the eliminated assembled operator.
template <int MODE, typename T, typename TX, typename TY>
__global__ void __launch_bounds__(256) mf_gather_kernel(Grid g, const T* __restrict__ E, const uint16_t* __restrict__ mask,
                                                        const TX* __restrict__ x, const T* __restrict__ b,
                                                        const T* __restrict__ Dinv, T omega, TY* __restrict__ y) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= g.Npad) return;
  if (n >= g.N) {
#pragma unroll
    for (int c = 0; c < 9; ++c) y[(int64_t)c * g.Npad + n] = (TY)0;
    return;
  }
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  T s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int a = 7; a >= 0; --a) {  // element (i - ax, j - ay, k - az) has this node as corner a
    const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - ((a >> 2) & 1);
    if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
    const int64_t e = ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez);
#pragma unroll
    for (int c = 0; c < 9; ++c) s[c] += E[eo_index(a, c, e)];
  }
  const unsigned mb = mask ? mask[n] : 0u;
  T r[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const T xv = (T)x[(int64_t)c * g.Npad + n];
    const T kx = ((mb >> c) & 1) ? xv : s[c];
    r[c] = (MODE == 0) ? kx : b[(int64_t)c * g.Npad + n] - kx;
  }
  if (MODE == 2) {
    const int t = n >> 6, l = n & 63;
    const T* Db = Dinv + (int64_t)t * Lay<T>::SLICE;
#pragma unroll
    for (int rr = 0; rr < 9; ++rr) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < 9; ++c) acc += Db[Lay<T>::off(rr * 9 + c, l)] * r[c];
      y[(int64_t)rr * g.Npad + n] = (TY)((T)x[(int64_t)rr * g.Npad + n] + omega * acc);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 9; ++c) y[(int64_t)c * g.Npad + n] = (TY)r[c];
  }
}

// Gauss-point Hessians of a slab (standard Gauss-point layout, entries
// 15.. of qp) -> matrix-free layout, FP64 and (optionally) FP32.  One thread
// per group of 4 consecutive entries of one (point, element), in the order of
// the matrix-free layout, so that every wavefront writes whole 1 KB spans.
__global__ void __launch_bounds__(256) mf_pack_kernel(Grid g, Chunk ck, const double* __restrict__ qp,
                                                      double* __restrict__ D64, float* __restrict__ D32,
                                                      int64_t eb0, int64_t neb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = neb * 64;  // threads per entry group
  const int k4 = (int)(t / per);
  if (k4 >= 30) return;
  const int64_t r = t - (int64_t)k4 * per;
  const int lane = (int)(r & 63);
  const int gp = lane >> 3;
  const int64_t e = (eb0 + (r >> 6)) * 8 + (lane & 7);
  const int64_t el = e - ck.e0;
  if (el < 0 || el >= ck.NEc) return;
  const int64_t stride = (int64_t)8 * ck.NEcpad;
  const double* src = qp + (int64_t)(15 + 4 * k4) * stride + (int64_t)gp * ck.NEcpad + el;
  double d[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) d[u] = src[(int64_t)u * stride];
  if (D64) {
    *reinterpret_cast<double2*>(D64 + mf_index<double>(g.NEpad, 4 * k4, gp, e)) = make_double2(d[0], d[1]);
    *reinterpret_cast<double2*>(D64 + mf_index<double>(g.NEpad, 4 * k4 + 2, gp, e)) = make_double2(d[2], d[3]);
  }
  if (D32)
    *reinterpret_cast<float4*>(D32 + mf_index<float>(g.NEpad, 4 * k4, gp, e)) =
        make_float4((float)d[0], (float)d[1], (float)d[2], (float)d[3]);
}

size_t mf_hessian_values(const Grid& g) { return (size_t)120 * 8 * g.NEpad; }

void launch_mf_pack(const Grid& g, const Chunk& ck, const double* qp, double* D64, float* D32, hipStream_t s) {
  const int64_t eb0 = ck.e0 / 8, eb1 = (ck.e0 + ck.NEc + 7) / 8;  // element groups of 8 touching the slab
  const int64_t n = 30 * (eb1 - eb0) * 64;
  mf_pack_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(g, ck, qp, D64, D32, eb0, eb1 - eb0);
}

template <typename TD, typename TX, typename T>
void launch_mf_element(const Grid& g, const TD* D, const TX* x, const uint16_t* mask, const DevCard* cd, T* E,
                       hipStream_t s) {
  const int64_t threads = (int64_t)g.NEpad * 8;  // NEpad is a multiple of 64: whole wavefronts
  constexpr int MINB = (sizeof(TD) == 8 && sizeof(TX) == 8) ? 2 : 3;  // all-FP64: no spills at 2
  mf_element_kernel<TD, TX, T, MINB><<<(int)((threads + 255) / 256), 256, 0, s>>>(g, D, x, mask, cd, E);
}

template <int MODE, typename T, typename TX, typename TY>
void launch_mf_gather(const Grid& g, const T* E, const uint16_t* mask, const TX* x, const T* b, const T* Dinv, T omega,
                      TY* y, hipStream_t s) {
  mf_gather_kernel<MODE, T, TX, TY><<<(g.Npad + 255) / 256, 256, 0, s>>>(g, E, mask, x, b, Dinv, omega, y);
}

template void launch_mf_element<float, float, float>(const Grid&, const float*, const float*, const uint16_t*,
                                                     const DevCard*, float*, hipStream_t);
template void launch_mf_element<double, float, double>(const Grid&, const double*, const float*, const uint16_t*,
                                                       const DevCard*, double*, hipStream_t);
template void launch_mf_element<double, double, double>(const Grid&, const double*, const double*, const uint16_t*,
                                                        const DevCard*, double*, hipStream_t);
template void launch_mf_gather<0, float, float, float>(const Grid&, const float*, const uint16_t*, const float*,
                                                       const float*, const float*, float, float*, hipStream_t);
template void launch_mf_gather<1, float, float, float>(const Grid&, const float*, const uint16_t*, const float*,
                                                       const float*, const float*, float, float*, hipStream_t);
template void launch_mf_gather<2, float, float, float>(const Grid&, const float*, const uint16_t*, const float*,
                                                       const float*, const float*, float, float*, hipStream_t);
template void launch_mf_gather<0, double, float, double>(const Grid&, const double*, const uint16_t*, const float*,
                                                         const double*, const double*, double, double*, hipStream_t);
template void launch_mf_gather<0, double, double, double>(const Grid&, const double*, const uint16_t*, const double*,
                                                          const double*, const double*, double, double*, hipStream_t);
template void launch_mf_gather<1, double, double, double>(const Grid&, const double*, const uint16_t*, const double*,
                                                          const double*, const double*, double, double*, hipStream_t);
template void launch_mf_gather<2, double, double, double>(const Grid&, const double*, const uint16_t*, const double*,
                                                          const double*, const double*, double, double*, hipStream_t);

}  // namespace mvpf
