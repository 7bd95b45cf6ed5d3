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
// 8 * element + j).  Lane j loads the 9 unknowns of corner j of its element
// and evaluates Gauss point j: since the Q1 shape functions and the 2x2x2
// points are tensor products, v_g follows from three one-dimensional
// interpolation stages over lane pairs (sum factorisation; lanes exchange
// values by DPP moves, xor 1, 2, 4), and the contributions B^T [w; z] go
// back to the corners through the transposed stages, so that lane j ends
// with the element's part for corner j.  The workgroup merges the parts of
// neighbouring elements along x that meet at a node and writes them to the
// element-output buffer (layout in common.h); a node gather sums its <= 4
// merged element rows in a fixed order and applies the epilogue (product,
// defect or damped point-block Jacobi update), so results are reproducible
// bit for bit.
//
// The lane layout (9 unknowns per corner, 15 local variables, 120 Hessian
// entries streamed as 30 16-byte vectors) is that of the six-variant card:
// a library built for another number of variants never enables the
// matrix-free level (its finest level is assembled like the others) and
// launches none of these kernels.
#include "common.h"

namespace mvpf {

constexpr double MGQ0 = 0.21132486540518711775;  // (1 - 1/sqrt 3) / 2
constexpr double MGQ1 = 0.78867513459481288225;

// Lane exchanges inside groups of 8 lanes by DPP (no LDS traffic): xor 1 and
// xor 2 are quad permutations; xor 4 is the half-row mirror (lane i <- 7 - i)
// followed by the quad reversal (i <- i ^ 3), since (7 - i) ^ 3 = i ^ 4.
template <int X, typename T>
__device__ __forceinline__ T lane_xor(T v) {
  if constexpr (X == 1) return dpp_t<0xB1>(v);       // quad_perm [1,0,3,2]
  else if constexpr (X == 2) return dpp_t<0x4E>(v);  // quad_perm [2,3,0,1]
  else return dpp_t<0x1B>(dpp_t<0x141>(v));          // row_half_mirror, then quad_perm [3,2,1,0]
}

// One direction of the trilinear interpolation at the Gauss points, by lane
// pairs (sum factorisation).  Each lane holds n values belonging to its node
// index bit b along this direction; with t = (partner's value) - (own value)
// it gets, at its Gauss coordinate q (the same bit selects q), the
// interpolated value s = own + qq t (qq = q for b = 0, 1 - q for b = 1) and,
// for the first nd values, the difference across the pair, d = sg t (sg = +1
// for b = 0, -1 for b = 1): the derivative along this direction on the unit
// reference cube.  The partner's value enters only through the subtraction,
// so the lane exchange folds into it (a DPP operand), and no lane selects
// are needed.
template <int X, typename T, int n, int nd>
__device__ __forceinline__ void interp_pair(const T (&in)[n], T qq, T sg, T (&s)[n], T (&d)[nd]) {
#pragma unroll
  for (int k = 0; k < n; ++k) {
    const T t = lane_xor<X>(in[k]) - in[k];
    s[k] = in[k] + qq * t;
    if (k < nd) d[k] = sg * t;
  }
}

// Transpose of interp_pair: a lane at Gauss coordinate q along this
// direction holds coefficients a (of the values) and bs = sb * b (of the
// derivatives, sb = -1 for node bit 0, +1 for bit 1: the sign is applied by
// the caller where b is formed); afterwards it holds, for its node bit, the
// sum over both Gauss points of a * phi(q) + b * phi', phi = 1 - q or q,
// phi' = -1 or +1.  Own part a mq + bs, partner's part a tq - bs (mq = 1 - q,
// tq = q for bit 0; mq = q, tq = 1 - q for bit 1); the exchange folds into the
// final addition.
template <int X, typename T, int n>
__device__ __forceinline__ void interp_pair_t(const T (&a)[n], const T (&bs)[n], T mq, T tq, T (&out)[n]) {
#pragma unroll
  for (int k = 0; k < n; ++k) {
    const T mine = a[k] * mq + bs[k];
    const T theirs = a[k] * tq - bs[k];
    out[k] = mine + lane_xor<X>(theirs);
  }
}

// elements per workgroup of the element kernels: 8, 16 or 32
constexpr int MF_MAX_EPW = 32;

// gradient-energy coefficient Mg[m][m2] in the arithmetic type
template <typename T>
__device__ __forceinline__ T mg_coef(const DevCard* __restrict__ cd, int m, int m2) {
  if constexpr (sizeof(T) == 4) return cd->Mg32[m][m2];
  else return cd->Mg[m][m2];
}

// E = element parts of K x_e (x masked on constrained dofs when mask != null).
// Lane = 8 * element + j: the lane loads the unknowns of corner j of its
// element and evaluates Gauss point j; the 15 local variables of every
// point come from three interpolation stages over lane pairs (x, y, z), and
// its contributions go back to the corners through the transposed stages
// (z, y, x), so that lane j ends with the element's part for corner j.
// SPARSE: x has few nonzero entries (the lifting of a prescribed increment):
// an element whose unknowns are all zero reads no Hessians; otherwise the
// Hessian loads are issued before the unknowns arrive.
// PF: Hessian vectors loaded ahead of the contraction (the rest are loaded
// PF vectors ahead of their use); MINB: minimum waves per SIMD the register
// budget is sized for.
template <typename TD, typename TX, typename T, int PF, bool SPARSE>
__device__ __forceinline__ void mf_element_body(const Grid& g, const TD* __restrict__ D, const TX* __restrict__ x,
                                                const uint16_t* __restrict__ mask, const DevCard* __restrict__ cd,
                                                T* __restrict__ E, int wg, int nb) {
  // workgroups are dealt to the 8 XCDs in turn: renumber them so that each
  // XCD takes one contiguous range of elements (corner unknowns shared by
  // neighbouring elements then hit that XCD's L2)
  const int xcd = wg & 7;
  const int bid = xcd * (nb >> 3) + min(xcd, nb & 7) + (wg >> 3);
  const int64_t t = (int64_t)bid * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int gp = lane & 7;
  const int64_t e = (t >> 6) * 8 + (lane >> 3);
  const bool active = e < g.NE;  // inactive lanes hold zeros and still take part in the exchanges
  const bool b0 = gp & 1, b1 = (gp >> 1) & 1, b2 = (gp >> 2) & 1;
  // per direction: qq (interpolation weight of the partner's difference) and
  // sg (sign of the derivative) of the forward stages; mq / tq (own and
  // partner's weight) and sb (derivative sign) of the transposed stages
  const T one = (T)1, lo = (T)MGQ0, hi = (T)MGQ1;
  const T qq0 = b0 ? one - hi : lo, qq1 = b1 ? one - hi : lo, qq2 = b2 ? one - hi : lo;
  const T sg0 = b0 ? -one : one, sg1 = b1 ? -one : one, sg2 = b2 ? -one : one;
  const T mq0 = b0 ? hi : one - lo, mq1 = b1 ? hi : one - lo, mq2 = b2 ? hi : one - lo;
  const T tq0 = b0 ? one - hi : lo, tq1 = b1 ? one - hi : lo, tq2 = b2 ? one - hi : lo;
  const T h = (T)g.h, c1 = (T)(0.125 * g.h);
  // the unknowns of corner gp
  T xa[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) xa[c] = 0;
  int node = 0;
  if (active) {
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    node = (ex + b0) + g.nnx * ((ey + b1) + g.nny * (ez + b2));
    const unsigned mb = mask ? mask[node] : 0u;
    TX xl[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) xl[c] = x[(int64_t)c * g.Npad + node];
#pragma unroll
    for (int c = 0; c < 9; ++c) xa[c] = ((mb >> c) & 1) ? (T)0 : (T)xl[c];
  }
  // Hessians of Gauss point gp (packed upper triangle, row-major p <= q),
  // 16-byte non-temporal loads (streamed once per product: x and the
  // element outputs stay in the caches)
  constexpr int V = 16 / (int)sizeof(TD);
  constexpr int NV = 120 / V;
  typedef TD VT __attribute__((ext_vector_type(V)));
  const VT* Dp = reinterpret_cast<const VT*>(D) + ((e >> 3) * NV * 64 + gp * 8 + (e & 7));
  constexpr int64_t ks = 64;
  VT dq[NV];
  if (!SPARSE && active) {
#pragma unroll
    for (int k = 0; k < PF; ++k) dq[k] = __builtin_nontemporal_load(Dp + k * ks);
  }
  // interpolation to Gauss point gp: x, then y, then z
  T s1[9], d1[9];
  interp_pair<1>(xa, qq0, sg0, s1, d1);
  T sd1[18], s2[18], d2[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) sd1[c] = s1[c], sd1[9 + c] = d1[c];
  interp_pair<2>(sd1, qq1, sg1, s2, d2);  // s2 = (value, d/dx) at (q0, q1); d2 = d/dy
  T sd2[27], s3[27], d3[9];
#pragma unroll
  for (int c = 0; c < 18; ++c) sd2[c] = s2[c];
#pragma unroll
  for (int c = 0; c < 9; ++c) sd2[18 + c] = d2[c];
  interp_pair<4>(sd2, qq2, sg2, s3, d3);  // s3 = (value, d/dx, d/dy); d3 = d/dz
  // v: reference gradients of u (3 x 3), h * eta (6); ge: reference gradients of eta
  T v[15], ge[18];
#pragma unroll
  for (int c = 0; c < 3; ++c) v[3 * c] = s3[9 + c], v[3 * c + 1] = s3[18 + c], v[3 * c + 2] = d3[c];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    v[9 + m] = h * s3[3 + m];
    ge[3 * m] = s3[12 + m], ge[3 * m + 1] = s3[21 + m], ge[3 * m + 2] = d3[3 + m];
  }
  // w = D v
  T w[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) w[k] = 0;
  bool load = active;
  if (SPARSE) {  // the element is zero iff the unknowns of its 8 corners (lanes) are
    bool nz = false;
#pragma unroll
    for (int c = 0; c < 9; ++c) nz = nz || xa[c] != (T)0;
    const unsigned long long bal = __ballot(nz);
    load = active && ((bal >> (lane & ~7)) & 0xFFull) != 0;
    if (load) {
#pragma unroll
      for (int k = 0; k < NV; ++k) dq[k] = __builtin_nontemporal_load(Dp + k * ks);
    }
  }
  if (load) {
#pragma unroll
    for (int p = 0, k = 0; p < 15; ++p)
#pragma unroll
      for (int qq = p; qq < 15; ++qq, ++k) {
        if (!SPARSE && k % V == 0 && k / V + PF < NV) dq[k / V + PF] = __builtin_nontemporal_load(Dp + (k / V + PF) * ks);
        const T d = (T)dq[k / V][k % V];
        w[p] += d * v[qq];
        if (qq != p) w[qq] += d * v[p];
      }
  }
  // gradient energy: z = (Mg (x) I) grad_ref eta
  T z[18];
#pragma unroll
  for (int m = 0; m < 6; ++m)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T sum = 0;
#pragma unroll
      for (int m2 = 0; m2 < 6; ++m2) sum += mg_coef<T>(cd, m, m2) * ge[3 * m2 + j];
      z[3 * m + j] = sum;
    }
  // coefficients of point gp: a = of the shape-function values, (bx, by, bz)
  // = of their reference derivatives, per component, each derivative
  // coefficient carrying the transposed stage's sign of its direction (the
  // x and y coefficients keep it through the z and y stages, whose lane
  // partners share the lane's x and y bits)
  const T cx = b0 ? c1 : -c1, cy = b1 ? c1 : -c1, cz = b2 ? c1 : -c1;
  T a3[27], bz[27];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a3[c] = 0, a3[9 + c] = cx * w[3 * c], a3[18 + c] = cy * w[3 * c + 1];
    bz[c] = cz * w[3 * c + 2];
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    a3[3 + m] = c1 * h * w[9 + m], a3[12 + m] = cx * z[3 * m], a3[21 + m] = cy * z[3 * m + 1];
    bz[3 + m] = cz * z[3 * m + 2];
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) bz[9 + c] = 0, bz[18 + c] = 0;
  // back to the corners: z (27 sums: value, x, y coefficients), then y, then x
  T r3[27];
  interp_pair_t<4>(a3, bz, mq2, tq2, r3);
  T a2[18], by[18], r2[18];
#pragma unroll
  for (int c = 0; c < 18; ++c) a2[c] = r3[c], by[c] = 0;
#pragma unroll
  for (int c = 0; c < 9; ++c) by[c] = r3[18 + c];
  interp_pair_t<2>(a2, by, mq1, tq1, r2);
  T a1[9], bx[9], out[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) a1[c] = r2[c], bx[c] = r2[9 + c];
  interp_pair_t<1>(a1, bx, mq0, tq0, out);
  // Element outputs through LDS: a lane holds corner gp's 9 values; staged
  // per stream (gp, c), the workgroup merges each element's left corners
  // with the right corners of its predecessor in the same row and stores
  // one contiguous, aligned run of each merged stream (whole 128-byte lines
  // at 32 elements in FP32), plus the right corners that no element of the
  // workgroup takes (its last element's, row ends).  Every lane of the
  // workgroup reaches the barrier.
  __shared__ T eo[72 * (MF_MAX_EPW + 1)];
  const int epw = blockDim.x >> 3;
  const int jw = threadIdx.x >> 3;  // element within the workgroup
#pragma unroll
  for (int c = 0; c < 9; ++c) eo[(gp * 9 + c) * (epw + 1) + jw] = out[c];
  __syncthreads();
  const int64_t ew = (int64_t)bid * epw;  // the workgroup's first element
  const int ex0 = (int)(ew % g.nx);
  T* __restrict__ W = E + mf_w_offset(g);
  T* __restrict__ Rr = E + mf_r_offset(g);
  for (int idx = threadIdx.x; idx < 36 * epw; idx += blockDim.x) {
    const int s = idx / epw, jj = idx - s * epw;  // merged stream s = 9 q + c
    const int64_t e = ew + jj;
    if (e >= g.NE) continue;
    const int q = s / 9, c = s - 9 * q;
    int ex = ex0 + jj;
    while (ex >= g.nx) ex -= g.nx;
    const T* left = eo + (18 * q + c) * (epw + 1);      // corner 2q
    const T* right = eo + (18 * q + 9 + c) * (epw + 1);  // corner 2q + 1
    T v = left[jj];
    if (jj > 0 && ex > 0) v = v + right[jj - 1];
    E[(int64_t)s * g.NEpad + e] = v;
    if (ex == g.nx - 1) Rr[(int64_t)s * mf_nr(g) + e / g.nx] = right[jj];
    else if (jj == epw - 1) W[(int64_t)s * mf_nw(g) + bid] = right[jj];
  }
}
template <typename TD, typename TX, typename T, int MINB, int PF, bool SPARSE>
__global__ void __launch_bounds__(256, MINB) mf_element_kernel(Grid g, const TD* __restrict__ D, const TX* __restrict__ x,
                                                               const uint16_t* __restrict__ mask,
                                                               const DevCard* __restrict__ cd, T* __restrict__ E) {
  mf_element_body<TD, TX, T, PF, SPARSE>(g, D, x, mask, cd, E, blockIdx.x, gridDim.x);
}

// Node gather with epilogue.  MODE 0: y = K x; 1: r = b - K x;
// 2: xo = x + omega Dinv (b - K x), Dinv packed symmetric (LaySym) in FP32,
// full (Lay) in FP64.  Constrained rows (mask) act as the identity, as in the
// eliminated assembled operator.  E: the element outputs of a launch with
// epw elements per workgroup; Cf: the contact face outputs, or null.
template <int MODE, typename T, typename TX, typename TY>
__device__ __forceinline__ void mf_gather_body(const Grid& g, const T* __restrict__ E, const T* __restrict__ Cf,
                                               int epw, const uint16_t* __restrict__ mask,
                                               const TX* __restrict__ x, const T* __restrict__ b,
                                               const T* __restrict__ Dinv, T omega, TY* __restrict__ y, int bid) {
  const int n = bid * 256 + threadIdx.x;
  if (n >= g.Npad) return;
  if (n >= g.N) {
#pragma unroll
    for (int c = 0; c < 9; ++c) y[(int64_t)c * g.Npad + n] = (TY)0;
    return;
  }
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  T s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const T* __restrict__ W = E + mf_w_offset(g);
  const T* __restrict__ Rr = E + mf_r_offset(g);
#pragma unroll
  for (int q = 3; q >= 0; --q) {  // element row r = (j - by) + ny (k - bz) holds this node at (by, bz)
    const int ey = j - (q & 1), ez = k - (q >> 1);
    if (ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
    const int64_t r = ey + (int64_t)g.ny * ez;
    T t[9];
    if (i < g.nx) {
      const int64_t e = i + g.nx * r;
#pragma unroll
      for (int c = 0; c < 9; ++c) t[c] = E[(int64_t)(9 * q + c) * g.NEpad + e];
      if (i > 0 && (e & (epw - 1)) == 0) {  // element e - 1 ended the previous workgroup
        const int64_t w = e / epw - 1;
#pragma unroll
        for (int c = 0; c < 9; ++c) t[c] = t[c] + W[(int64_t)(9 * q + c) * mf_nw(g) + w];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) t[c] = Rr[(int64_t)(9 * q + c) * mf_nr(g) + r];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) s[c] += t[c];
  }
  if (Cf && k == g.nz) {  // penalty contact: the top faces around the node
    const int64_t nf = mf_nf(g);
#pragma unroll
    for (int a = 3; a >= 0; --a) {
      const int fi = i - (a & 1), fj = j - (a >> 1);
      if (fi < 0 || fi >= g.nx || fj < 0 || fj >= g.ny) continue;
      const int64_t f = fi + (int64_t)g.nx * fj;
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c] += Cf[(3 * a + c) * nf + f];
    }
  }
  const unsigned mb = mask ? mask[n] : 0u;
  T r[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const T xv = (T)x[(int64_t)c * g.Npad + n];
    const T kx = ((mb >> c) & 1) ? xv : s[c];
    r[c] = (MODE == 0) ? kx : b[(int64_t)c * g.Npad + n] - kx;
  }
  if (MODE == 2 && sizeof(T) == 4) {  // FP32: the packed upper triangles of the symmetric block inverses
    const int t = n >> 6, l = n & 63;
    const T* Db = Dinv + (int64_t)t * LaySym<T>::SLICE;
    T dv[NSYM];
#pragma unroll
    for (int e = 0; e < NSYM; ++e) dv[e] = Db[LaySym<T>::off(e, l)];
#pragma unroll
    for (int rr = 0; rr < 9; ++rr) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < 9; ++c) acc += dv[sym_index(rr, c)] * r[c];
      y[(int64_t)rr * g.Npad + n] = (TY)((T)x[(int64_t)rr * g.Npad + n] + omega * acc);
    }
  } else if (MODE == 2) {
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
template <int MODE, typename T, typename TX, typename TY>
__global__ void __launch_bounds__(256) mf_gather_kernel(Grid g, const T* __restrict__ E, const T* __restrict__ Cf,
                                                        int epw, const uint16_t* __restrict__ mask,
                                                        const TX* __restrict__ x, const T* __restrict__ b,
                                                        const T* __restrict__ Dinv, T omega, TY* __restrict__ y) {
  mf_gather_body<MODE, T, TX, TY>(g, E, Cf, epw, mask, x, b, Dinv, omega, y, blockIdx.x);
}

// Gauss-point Hessians of a slab (standard Gauss-point layout, entries
// 15.. of qp) -> matrix-free layout, FP64 and (optionally) FP32.  One thread
// per group of 4 consecutive entries of one (point, element), in the order of
// the matrix-free layout, so that every wavefront writes whole 1 KB spans.
__device__ __forceinline__ void mf_pack_body(const Grid& g, const Chunk& ck, const double* __restrict__ qp,
                                             double* __restrict__ D64, float* __restrict__ D32, int64_t eb0,
                                             int64_t neb, int bid) {
  const int64_t t = (int64_t)bid * 256 + threadIdx.x;
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

__global__ void __launch_bounds__(256) mf_pack_kernel(Grid g, Chunk ck, const double* __restrict__ qp,
                                                      double* __restrict__ D64, float* __restrict__ D32,
                                                      int64_t eb0, int64_t neb) {
  mf_pack_body(g, ck, qp, D64, D32, eb0, neb, blockIdx.x);
}
__global__ void __launch_bounds__(256) mf_pack_batch(const AJob* __restrict__ jobs, int njobs) {
  int bid;
  const AJob& j = find_job(jobs, njobs, bid);
  mf_pack_body(j.g, j.ck, j.qp, j.D64, j.D32, j.eb0, j.neb, bid);
}
void launch_mf_pack_batch(const AJob* jobs, int njobs, int blocks, hipStream_t s) {
  if (!MF_AVAILABLE) return;
  mf_pack_batch<<<blocks, 256, 0, s>>>(jobs, njobs);
}
int mf_pack_job_blocks(AJob& j) {
  j.eb0 = j.ck.e0 / 8;
  j.neb = (j.ck.e0 + j.ck.NEc + 7) / 8 - j.eb0;
  return (int)((30 * j.neb * 64 + 255) / 256);
}

size_t mf_hessian_values(const Grid& g) { return MF_AVAILABLE ? (size_t)120 * 8 * g.NEpad : 0; }

void launch_mf_pack(const Grid& g, const Chunk& ck, const double* qp, double* D64, float* D32, hipStream_t s) {
  if (!MF_AVAILABLE) return;
  const int64_t eb0 = ck.e0 / 8, eb1 = (ck.e0 + ck.NEc + 7) / 8;  // element groups of 8 touching the slab
  const int64_t n = 30 * (eb1 - eb0) * 64;
  mf_pack_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(g, ck, qp, D64, D32, eb0, eb1 - eb0);
}

// Register budgets (measured equal within 1 % for prefetch depths 12 ... 30
// at 2 ... 4 waves per SIMD): FP32 Hessians 20 vectors ahead at >= 3 waves
// per SIMD, FP64 16 ahead at >= 2.
constexpr int MF_PF32 = 20, MF_MINB32 = 3, MF_PF64 = 16, MF_MINB64 = 2;
template <typename TD, typename TX, typename T>
void launch_mf_element(const Grid& g, const TD* D, const TX* x, const uint16_t* mask, const DevCard* cd, T* E,
                       hipStream_t s, bool sparse_x, int elems_per_wg) {
  if constexpr (!MF_AVAILABLE) return;
  const int64_t threads = (int64_t)g.NEpad * 8;  // NEpad is a multiple of 64: whole wavefronts
  constexpr bool f64 = sizeof(TD) == 8;
  constexpr int MINB = f64 ? MF_MINB64 : MF_MINB32, PF = f64 ? MF_PF64 : MF_PF32;
  const int wg = 8 * mf_epw_of(elems_per_wg);  // divides threads
  const int blocks = (int)(threads / wg);
  if (sparse_x)
    mf_element_kernel<TD, TX, T, MINB, PF, true><<<blocks, wg, 0, s>>>(g, D, x, mask, cd, E);
  else
    mf_element_kernel<TD, TX, T, MINB, PF, false><<<blocks, wg, 0, s>>>(g, D, x, mask, cd, E);
}

template <int MODE, typename T, typename TX, typename TY>
void launch_mf_gather(const Grid& g, const T* E, bool contact, int elems_per_wg, const uint16_t* mask, const TX* x,
                      const T* b, const T* Dinv, T omega, TY* y, hipStream_t s) {
  if constexpr (!MF_AVAILABLE) return;
  mf_gather_kernel<MODE, T, TX, TY><<<(g.Npad + 255) / 256, 256, 0, s>>>(
      g, E, contact ? E + mf_cf_offset(g) : nullptr, mf_epw_of(elems_per_wg), mask, x, b, Dinv, omega, y);
}

template void launch_mf_element<float, float, float>(const Grid&, const float*, const float*, const uint16_t*,
                                                     const DevCard*, float*, hipStream_t, bool, int);
template void launch_mf_element<double, float, double>(const Grid&, const double*, const float*, const uint16_t*,
                                                       const DevCard*, double*, hipStream_t, bool, int);
template void launch_mf_element<double, double, double>(const Grid&, const double*, const double*, const uint16_t*,
                                                        const DevCard*, double*, hipStream_t, bool, int);
template void launch_mf_gather<0, float, float, float>(const Grid&, const float*, bool, int, const uint16_t*,
                                                       const float*, const float*, const float*, float, float*,
                                                       hipStream_t);
template void launch_mf_gather<1, float, float, float>(const Grid&, const float*, bool, int, const uint16_t*,
                                                       const float*, const float*, const float*, float, float*,
                                                       hipStream_t);
template void launch_mf_gather<2, float, float, float>(const Grid&, const float*, bool, int, const uint16_t*,
                                                       const float*, const float*, const float*, float, float*,
                                                       hipStream_t);
template void launch_mf_gather<0, double, float, double>(const Grid&, const double*, bool, int, const uint16_t*,
                                                         const float*, const double*, const double*, double, double*,
                                                         hipStream_t);
template void launch_mf_gather<0, double, double, double>(const Grid&, const double*, bool, int, const uint16_t*,
                                                          const double*, const double*, const double*, double,
                                                          double*, hipStream_t);
template void launch_mf_gather<1, double, double, double>(const Grid&, const double*, bool, int, const uint16_t*,
                                                          const double*, const double*, const double*, double,
                                                          double*, hipStream_t);
template void launch_mf_gather<2, double, double, double>(const Grid&, const double*, bool, int, const uint16_t*,
                                                          const double*, const double*, const double*, double,
                                                          double*, hipStream_t);

// ---- batched launches (FP32 or FP64 smoothing on matrix-free finest levels) ----
template <typename T, int MINB, int PF>
__global__ void __launch_bounds__(256, MINB) mf_element_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  mf_element_body<T, T, T, PF, false>(j.g, (const T*)j.A, (const T*)j.x, j.mask, j.cd, (T*)j.C, bid, j.nblk);
}
template <int MODE, typename T>
__global__ void __launch_bounds__(256) mf_gather_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  mf_gather_body<MODE, T, T, T>(j.g, (const T*)j.C, j.contact ? (const T*)j.C + mf_cf_offset(j.g) : nullptr, j.epw,
                                j.mask, (const T*)j.x, (const T*)j.b, (const T*)j.D, (T)j.omega,
                                (T*)j.y, bid);
}
template <typename T>
void launch_mf_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s, int threads) {
  if constexpr (!MF_AVAILABLE) return;
  constexpr bool f64 = sizeof(T) == 8;
  if (op == BOP_MF_ELEMENT)
    mf_element_batch<T, f64 ? MF_MINB64 : MF_MINB32, f64 ? MF_PF64 : MF_PF32><<<blocks, threads, 0, s>>>(jobs, njobs);
  else if (op == BOP_MF_GATHER_PBJ)
    mf_gather_batch<2, T><<<blocks, 256, 0, s>>>(jobs, njobs);
  else if (op == BOP_MF_GATHER_DEFECT)
    mf_gather_batch<1, T><<<blocks, 256, 0, s>>>(jobs, njobs);
}
template void launch_mf_batch<float>(int, const BJob*, int, int, hipStream_t, int);
template void launch_mf_batch<double>(int, const BJob*, int, int, hipStream_t, int);
// element kernels: threads (64, 128 or 256) divide the 8 NEpad lanes exactly
int mf_job_blocks(int op, const Grid& g, int threads) {
  return (op == BOP_MF_ELEMENT || op == BOP_MF_OUTER_ELEMENT) ? (int)((int64_t)g.NEpad * 8 / threads)
                                                             : (g.Npad + 255) / 256;
}

// batched FGMRES operator product on matrix-free finest levels: FP64
// Hessians, input z of type TZ (the preconditioned vector), FP64 output
template <typename TZ>
__global__ void __launch_bounds__(256, MF_MINB64) mf_outer_element_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  mf_element_body<double, TZ, double, MF_PF64, false>(j.g, (const double*)j.A, (const TZ*)j.x, j.mask, j.cd,
                                                      (double*)j.C, bid, j.nblk);
}
template <typename TZ>
__global__ void __launch_bounds__(256) mf_outer_gather_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  mf_gather_body<0, double, TZ, double>(j.g, (const double*)j.C,
                                        j.contact ? (const double*)j.C + mf_cf_offset(j.g) : nullptr, j.epw, j.mask,
                                        (const TZ*)j.x, nullptr, nullptr, 0.0,
                                        (double*)j.y, bid);
}
template <typename TZ>
void launch_mf_outer_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s, int threads) {
  if constexpr (!MF_AVAILABLE) return;
  if (op == BOP_MF_OUTER_ELEMENT)
    mf_outer_element_batch<TZ><<<blocks, threads, 0, s>>>(jobs, njobs);
  else if (op == BOP_MF_OUTER_GATHER)
    mf_outer_gather_batch<TZ><<<blocks, 256, 0, s>>>(jobs, njobs);
}
template void launch_mf_outer_batch<float>(int, const BJob*, int, int, hipStream_t, int);
template void launch_mf_outer_batch<double>(int, const BJob*, int, int, hipStream_t, int);

}  // namespace mvpf
