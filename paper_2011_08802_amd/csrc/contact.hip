// Frictionless penalty contact of the top face with a rigid spherical
// indenter (Sec. 2.4, Eqs. Ngap and PenPot).
//
// On each top face u is bilinear in its four nodes and the surface integral
// uses 2x2 Gauss points (weights h^2/4).  At a point with current position
// x = X + u, r = |x - c|, the gap is g = r - R and the sphere's normal
// n = (x - c)/r.  Active points (g < 0) contribute
//   energy     1/2 eps g^2
//   force      eps g n N_a                                   (residual rows)
//   stiffness  N_a N_b eps [n n^T + g/r (I - n n^T)]         (u-u blocks)
//   load       eps g n_z  (the force conjugate to the indenter depth)
// The residual and the load are gathered per node / in one workgroup in a
// fixed order, the stiffness is added to the element matrices of the top
// element layer before their gather, so every result is reproducible bit
// for bit.
#include "common.h"

namespace mvpf {

namespace {

constexpr double GQ0 = 0.21132486540518711775;  // (1 - 1/sqrt 3) / 2
constexpr double GQ1 = 0.78867513459481288225;  // (1 + 1/sqrt 3) / 2

// Gauss point q (0..3) of top face (fi, fj): shape values of the face's
// nodes a = ax + 2 ay, the point's current position x and the gap data.
struct FacePoint {
  double N[4];
  double d[3];  // x - c
  double r, gap;
};

__device__ __forceinline__ void face_point(const Grid& g, const Sphere& s, const double* __restrict__ state, int fi,
                                           int fj, int q, FacePoint& fp) {
  const double xi = (q & 1) ? GQ1 : GQ0, et = (q & 2) ? GQ1 : GQ0;
  fp.N[0] = (1.0 - xi) * (1.0 - et);
  fp.N[1] = xi * (1.0 - et);
  fp.N[2] = (1.0 - xi) * et;
  fp.N[3] = xi * et;
  double x[3] = {(fi + xi) * g.h, (fj + et) * g.h, g.nz * g.h};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int node = (fi + (a & 1)) + g.nnx * ((fj + (a >> 1)) + g.nny * g.nz);
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] += fp.N[a] * state[(int64_t)c * g.Npad + node];
  }
  fp.d[0] = x[0] - s.cx;
  fp.d[1] = x[1] - s.cy;
  fp.d[2] = x[2] - s.cz;
  fp.r = sqrt(fp.d[0] * fp.d[0] + fp.d[1] * fp.d[1] + fp.d[2] * fp.d[2]);
  fp.gap = fp.r - s.R;
}

// R += contact force rows of the top nodes (one thread per top node)
__global__ void __launch_bounds__(256) contact_residual_kernel(Grid g, Sphere s, const double* __restrict__ state,
                                                               double* __restrict__ R) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= g.nnx * g.nny) return;
  const int i = t % g.nnx, j = t / g.nnx;
  const double w = 0.25 * g.h * g.h * s.eps;
  double f[3] = {0.0, 0.0, 0.0};
  for (int fj = j - 1; fj <= j; ++fj)
    for (int fi = i - 1; fi <= i; ++fi) {
      if (fi < 0 || fi >= g.nx || fj < 0 || fj >= g.ny) continue;
      const int a = (i - fi) + 2 * (j - fj);
      for (int q = 0; q < 4; ++q) {
        FacePoint fp;
        face_point(g, s, state, fi, fj, q, fp);
        if (fp.gap < 0.0) {
          const double coef = w * fp.gap * fp.N[a] / fp.r;
#pragma unroll
          for (int c = 0; c < 3; ++c) f[c] += coef * fp.d[c];
        }
      }
    }
  const int node = t + g.nnx * g.nny * g.nz;
#pragma unroll
  for (int c = 0; c < 3; ++c) R[(int64_t)c * g.Npad + node] += f[c];
}

// Element matrices of the top element layer += face stiffness (one thread per
// top element; element-local nodes 4..7 are the face's nodes 0..3).
__global__ void __launch_bounds__(256) contact_element_kernel(Grid g, Chunk ck, Sphere s,
                                                              const double* __restrict__ state,
                                                              double* __restrict__ E, bool diag_only) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= g.nx * g.ny) return;
  const int fi = t % g.nx, fj = t / g.nx;
  const int64_t el = (int64_t)(g.nz - 1) * g.nx * g.ny + t - ck.e0;  // in the chunk (checked by the host)
  const double w = 0.25 * g.h * g.h * s.eps;
  double A[4][6];   // per Gauss point: w eps [n n^T + g/r (I - n n^T)], symmetric components
  double N[4][4];
  bool any = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    FacePoint fp;
    face_point(g, s, state, fi, fj, q, fp);
#pragma unroll
    for (int a = 0; a < 4; ++a) N[q][a] = fp.N[a];
    const bool act = fp.gap < 0.0;
    any = any || act;
    const double ir = 1.0 / fp.r;
    const double n0 = fp.d[0] * ir, n1 = fp.d[1] * ir, n2 = fp.d[2] * ir;
    const double gr = fp.gap * ir;
    const double cn = act ? w * (1.0 - gr) : 0.0, ci = act ? w * gr : 0.0;
    A[q][0] = cn * n0 * n0 + ci;
    A[q][1] = cn * n1 * n1 + ci;
    A[q][2] = cn * n2 * n2 + ci;
    A[q][3] = cn * n1 * n2;
    A[q][4] = cn * n0 * n2;
    A[q][5] = cn * n0 * n1;
  }
  if (!any) return;
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < (diag_only ? a + 1 : 4); ++b) {
      double K[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double nn = N[q][a] * N[q][b];
#pragma unroll
        for (int v = 0; v < 6; ++v) K[v] += nn * A[q][v];
      }
      const int p = pair_index(4 + a, 4 + b);
      double* Ep = E + (int64_t)p * NBLK * ck.NEcpad + el;
#pragma unroll
      for (int i3 = 0; i3 < 3; ++i3)
#pragma unroll
        for (int k3 = 0; k3 < 3; ++k3) Ep[(int64_t)(NDOF * i3 + k3) * ck.NEcpad] += K[SI(i3, k3)];
    }
}

// Face stiffness times x for the top faces (matrix-free finest level), into
// the contact part of the element-output buffer: one thread per top face,
// face corner a = bx + 2 by, x masked on constrained dofs; zeros where no
// face point is in contact.  The indenter is read from device memory, so a
// captured graph follows its depth.
template <typename T, typename TX>
__global__ void __launch_bounds__(256) contact_apply_kernel(Grid g, const Sphere* __restrict__ sp,
                                                            const double* __restrict__ state,
                                                            const uint16_t* __restrict__ mask,
                                                            const TX* __restrict__ x, T* __restrict__ E) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= g.nx * g.ny) return;
  const Sphere s = *sp;
  const int fi = t % g.nx, fj = t / g.nx;
  const double w = 0.25 * g.h * g.h * s.eps;
  double xb[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int node = (fi + (a & 1)) + g.nnx * ((fj + (a >> 1)) + g.nny * g.nz);
    const unsigned mb = mask ? mask[node] : 0u;
#pragma unroll
    for (int c = 0; c < 3; ++c) xb[a][c] = ((mb >> c) & 1) ? 0.0 : (double)x[(int64_t)c * g.Npad + node];
  }
  double out[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int q = 0; q < 4; ++q) {
    FacePoint fp;
    face_point(g, s, state, fi, fj, q, fp);
    if (!(fp.gap < 0.0)) continue;
    const double ir = 1.0 / fp.r;
    const double n[3] = {fp.d[0] * ir, fp.d[1] * ir, fp.d[2] * ir};
    const double gr = fp.gap * ir;
    double tq[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) tq[c] += fp.N[b] * xb[b][c];
    const double nt = n[0] * tq[0] + n[1] * tq[1] + n[2] * tq[2];
    // A t = w [(1 - g/r) n (n . t) + g/r t]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double at = w * ((1.0 - gr) * n[c] * nt + gr * tq[c]);
#pragma unroll
      for (int a = 0; a < 4; ++a) out[a][c] += fp.N[a] * at;
    }
  }
  T* __restrict__ Cf = E + mf_cf_offset(g);
  const int64_t nf = mf_nf(g);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) Cf[(3 * a + c) * nf + t] = (T)out[a][c];
}

// P = sum over active face points of w eps g n_z (one workgroup, fixed order)
__global__ void __launch_bounds__(256) contact_load_kernel(Grid g, Sphere s, const double* __restrict__ state,
                                                           double* __restrict__ out) {
  __shared__ double red[256];
  const double w = 0.25 * g.h * g.h * s.eps;
  double acc = 0.0;
  for (int f = threadIdx.x; f < g.nx * g.ny; f += 256) {
    const int fi = f % g.nx, fj = f / g.nx;
    for (int q = 0; q < 4; ++q) {
      FacePoint fp;
      face_point(g, s, state, fi, fj, q, fp);
      if (fp.gap < 0.0) acc += w * fp.gap * fp.d[2] / fp.r;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

Sphere make_sphere(const Grid& g, const mvpf_loading& ld, double depth) {
  Sphere s;
  s.cx = 0.5 * g.nx * g.h;
  s.cy = 0.5 * g.ny * g.h;
  s.cz = g.nz * g.h + ld.radius - depth;
  s.R = ld.radius;
  s.eps = ld.eps_n;
  return s;
}

void launch_contact_residual(const Grid& g, const Sphere& s, const double* state, double* R, hipStream_t st) {
  const int n = g.nnx * g.nny;
  contact_residual_kernel<<<(n + 255) / 256, 256, 0, st>>>(g, s, state, R);
}

bool chunk_has_top_layer(const Grid& g, const Chunk& ck) {
  return ck.e0 <= (int64_t)(g.nz - 1) * g.nx * g.ny && ck.e0 + ck.NEc == (int64_t)g.NE;
}

void launch_contact_element(const Grid& g, const Chunk& ck, const Sphere& s, const double* state, double* elem,
                            hipStream_t st, bool diag_only) {
  if (!chunk_has_top_layer(g, ck)) return;
  const int n = g.nx * g.ny;
  contact_element_kernel<<<(n + 255) / 256, 256, 0, st>>>(g, ck, s, state, elem, diag_only);
}

void launch_contact_load(const Grid& g, const Sphere& s, const double* state, double* out, hipStream_t st) {
  contact_load_kernel<<<1, 256, 0, st>>>(g, s, state, out);
}

template <typename T, typename TX>
void launch_contact_apply(const Grid& g, const Sphere* sp, const double* state, const uint16_t* mask, const TX* x, T* E,
                          hipStream_t st) {
  const int n = g.nx * g.ny;
  contact_apply_kernel<T, TX><<<(n + 255) / 256, 256, 0, st>>>(g, sp, state, mask, x, E);
}
template void launch_contact_apply<float, float>(const Grid&, const Sphere*, const double*, const uint16_t*,
                                                 const float*, float*, hipStream_t);
template void launch_contact_apply<double, float>(const Grid&, const Sphere*, const double*, const uint16_t*,
                                                  const float*, double*, hipStream_t);
template void launch_contact_apply<double, double>(const Grid&, const Sphere*, const double*, const uint16_t*,
                                                   const double*, double*, hipStream_t);

}  // namespace mvpf
