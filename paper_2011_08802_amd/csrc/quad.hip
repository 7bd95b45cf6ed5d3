// Quadrature and assembly kernels (Sec. 3.3-3.4): residual R = dPi/dU and
// tangent K = d^2 Pi / dU^2 of the discrete potential on Q1 hexahedra with
// 2x2x2 Gauss points, assembled without atomics:
//   1. qp_kernel: one thread per (Gauss point, element) evaluates the local
//      gradient (and Hessian) of the density and stores it (SoA, coalesced);
//   2. residual_gather: one thread per node sums its <= 8 elements;
//   3. element_matrix: element blocks for the 36 node pairs a <= b, with the
//      Gauss-point Hessians shared through LDS;
//   4. jacobian_gather: one thread per (node row, stored stencil block) sums
//      the <= 8 element blocks of the elements containing both nodes and
//      writes the 9x9 block into the tiled half-stencil layout.
// Summation order is fixed, so results are bitwise reproducible.
#include "common.h"

namespace mvpf {

// Gauss abscissae on [0,1]: (1 -+ 1/sqrt(3)) / 2
constexpr double GQ0 = 0.21132486540518711775;
constexpr double GQ1 = 0.78867513459481288225;

struct Shape {
  double N;
  double dN[3];  // reference-cube derivatives (divide by h for physical)
};

__device__ __forceinline__ Shape shape(int g, int a) {
  const double x[3] = {(g & 1) ? GQ1 : GQ0, (g & 2) ? GQ1 : GQ0, (g & 4) ? GQ1 : GQ0};
  double f[3], df[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool bit = (a >> d) & 1;
    f[d] = bit ? x[d] : 1.0 - x[d];
    df[d] = bit ? 1.0 : -1.0;
  }
  Shape s;
  s.N = f[0] * f[1] * f[2];
  s.dN[0] = df[0] * f[1] * f[2];
  s.dN[1] = f[0] * df[1] * f[2];
  s.dN[2] = f[0] * f[1] * df[2];
  return s;
}

// reference Laplacian 1/8 sum_g dN_a(g) . dN_b(g)  (element matrix = h * this)
__device__ __forceinline__ double lap_ref(int a, int b) {
  double s = 0.0;
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    const Shape sa = shape(g, a), sb = shape(g, b);
    s += sa.dN[0] * sb.dN[0] + sa.dN[1] * sb.dN[1] + sa.dN[2] * sb.dN[2];
  }
  return 0.125 * s;
}

template <bool HESS, int PD, int MIX>
__device__ __forceinline__ void qp_body(const Grid& g, const Chunk& ck, const double* __restrict__ state,
                                        const DevCard* __restrict__ cd, double* __restrict__ qp, int bid) {
  const int64_t tid = (int64_t)bid * 128 + threadIdx.x;
  const int gp = (int)(tid / ck.NEcpad);
  const int el = (int)(tid - (int64_t)gp * ck.NEcpad);
  if (gp >= 8 || el >= ck.NEc) return;
  const int64_t e = ck.e0 + el;
  const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
  const double ih = 1.0 / g.h;
  double F[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double eh[NV], ehn[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) eh[k] = ehn[k] = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int node = (ex + (a & 1)) + g.nnx * ((ey + ((a >> 1) & 1)) + g.nny * (ez + ((a >> 2) & 1)));
    const Shape s = shape(gp, a);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double u = state[(int64_t)i * g.Npad + node];
#pragma unroll
      for (int j = 0; j < 3; ++j) F[3 * i + j] += u * s.dN[j] * ih;
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      eh[k] += s.N * state[(int64_t)(3 + k) * g.Npad + node];
      ehn[k] += s.N * state[(int64_t)(3 + NV + k) * g.Npad + node];
    }
  }
  const int64_t stride = (int64_t)8 * ck.NEcpad;
  double* out = qp + (int64_t)gp * ck.NEcpad + el;
  double gr[NQ];
  if (HESS) {
    local_hessian<PD, MIX>(F, eh, ehn, *cd, gr, out + (int64_t)NQ * stride, stride);
  } else {
    local_gradient<PD, MIX>(F, eh, ehn, *cd, gr);
  }
#pragma unroll
  for (int c = 0; c < NQ; ++c) out[(int64_t)c * stride] = gr[c];
}
template <bool HESS, int PD, int MIX>
__global__ void __launch_bounds__(128) qp_kernel(Grid g, Chunk ck, const double* __restrict__ state,
                                                 const DevCard* __restrict__ cd, double* __restrict__ qp) {
  qp_body<HESS, PD, MIX>(g, ck, state, cd, qp, blockIdx.x);
}

template <int PD, int MIX>
void launch_qp_order(const Grid& g, const Chunk& ck, const double* state, const DevCard* cd, double* qp, bool hess,
                     hipStream_t s) {
  const int64_t n = (int64_t)8 * ck.NEcpad;
  const int bs = 128;
  const int nb = (int)((n + bs - 1) / bs);
  if (hess)
    qp_kernel<true, PD, MIX><<<nb, bs, 0, s>>>(g, ck, state, cd, qp);
  else
    qp_kernel<false, PD, MIX><<<nb, bs, 0, s>>>(g, ck, state, cd, qp);
}

// pade: 11, 22 or 33; mixing: MVPF_MIX_LINEAR or MVPF_MIX_LOG (validated at creation)
void launch_qp(const Grid& g, const Chunk& ck, const double* state, const DevCard* cd, int pade, int mixing,
               double* qp, bool hess, hipStream_t s) {
  if (mixing == MVPF_MIX_LOG) {
    switch (pade) {
      case 11: launch_qp_order<11, 1>(g, ck, state, cd, qp, hess, s); break;
      case 33: launch_qp_order<33, 1>(g, ck, state, cd, qp, hess, s); break;
      default: launch_qp_order<22, 1>(g, ck, state, cd, qp, hess, s); break;
    }
    return;
  }
  switch (pade) {
    case 11: launch_qp_order<11, 0>(g, ck, state, cd, qp, hess, s); break;
    case 33: launch_qp_order<33, 0>(g, ck, state, cd, qp, hess, s); break;
    default: launch_qp_order<22, 0>(g, ck, state, cd, qp, hess, s); break;
  }
}

__device__ __forceinline__ void residual_gather_body(const Grid& g, const Chunk& ck, const double* __restrict__ state,
                                                     const double* __restrict__ qp, const DevCard* __restrict__ cd,
                                                     double* __restrict__ R, int bid) {
  const int n = ck.n0 + bid * 256 + threadIdx.x;
  if (n >= ck.n1 || n >= g.Npad) return;
  double r[NDOF];
#pragma unroll
  for (int c = 0; c < NDOF; ++c) r[c] = 0.0;
  if (n < g.N) {
    const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
    const double cu = g.h * g.h * 0.125, ce = g.h * g.h * g.h * 0.125;
    const int64_t stride = (int64_t)8 * ck.NEcpad;
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const int ex = i - ax, ey = j - ay, ez = k - az;
      if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
      const int64_t el = ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez) - ck.e0;  // in [0, NEc) by construction
#pragma unroll
      for (int gp = 0; gp < 8; ++gp) {
        const Shape s = shape(gp, a);
        const double* q = qp + (int64_t)gp * ck.NEcpad + el;
#pragma unroll
        for (int i3 = 0; i3 < 3; ++i3)
          r[i3] += cu * (s.dN[0] * q[(3 * i3 + 0) * stride] + s.dN[1] * q[(3 * i3 + 1) * stride] +
                         s.dN[2] * q[(3 * i3 + 2) * stride]);
#pragma unroll
        for (int m = 0; m < NV; ++m) r[3 + m] += ce * s.N * q[(9 + m) * stride];
      }
      // gradient energy 1/2 Mg_kl grad eta_k . grad eta_l: h * Lap_ab * Mg * eta_b
      for (int b = 0; b < 8; ++b) {
        const int nb = (ex + (b & 1)) + g.nnx * ((ey + ((b >> 1) & 1)) + g.nny * (ez + ((b >> 2) & 1)));
        const double lap = g.h * lap_ref(a, b);
        double eb[NV];
#pragma unroll
        for (int l = 0; l < NV; ++l) eb[l] = state[(int64_t)(3 + l) * g.Npad + nb];
#pragma unroll
        for (int m = 0; m < NV; ++m) {
          double s2 = 0.0;
#pragma unroll
          for (int l = 0; l < NV; ++l) s2 += cd->Mg[m][l] * eb[l];
          r[3 + m] += lap * s2;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NDOF; ++c) R[(int64_t)c * g.Npad + n] = r[c];
}
__global__ void __launch_bounds__(256) residual_gather_kernel(Grid g, Chunk ck, const double* __restrict__ state,
                                                              const double* __restrict__ qp,
                                                              const DevCard* __restrict__ cd,
                                                              double* __restrict__ R) {
  residual_gather_body(g, ck, state, qp, cd, R, blockIdx.x);
}

void launch_residual_gather(const Grid& g, const Chunk& ck, const double* state, const double* qp, const DevCard* cd,
                            double* R, hipStream_t s) {
  residual_gather_kernel<<<(ck.n1 - ck.n0 + 255) / 256, 256, 0, s>>>(g, ck, state, qp, cd, R);
}


// Element matrices K_e = sum_g w_g B_g^T D_g B_g + h Lap (x) Mg for the 36
// node pairs a <= b.  A workgroup of EM_WAVES wavefronts covers 64
// consecutive elements and EM_WAVES pairs; the Gauss-point Hessians of those
// elements are staged once per Gauss point in LDS and shared by the
// wavefronts (wave = pair, lane = element), so each Hessian is read from L2
// 36 / EM_WAVES times in total.  Four waves leave room for the NDOF^2 FP64
// accumulators in registers (81 for N = 6: no spills).
constexpr int EM_WAVES = 4;
// workgroups per CU the registers are budgeted for (the staged Hessians of
// 15 unknowns per node take 116 KB of LDS: one workgroup per CU)
constexpr int EM_MINB = NHP_PAD * 64 * 8 <= 80 * 1024 ? 2 : 1;

// npair = NPAIR: all 36 pairs; npair = 8: the diagonal pairs (a, a) only.
__device__ __forceinline__ void element_matrix_body(const Grid& g, const Chunk& ck, const double* __restrict__ qp,
                                                    const DevCard* __restrict__ cd, double* __restrict__ E, int npair,
                                                    int bid, int nblk) {
  __shared__ double Ds[NHP_PAD * 64];
  // the NPAIR / EM_WAVES pair chunks of one element group are consecutive
  // logical blocks on one XCD, so the group's Hessians are read from HBM once
  // and then hit that XCD's L2
  const int groups = ck.NEcpad / 64;
  const int chunks = npair / EM_WAVES;
  const int Lb = xcd_logical(bid, nblk);
  if (Lb >= groups * chunks) return;  // uniform; before any barrier
  const int eg = Lb / chunks;
  const int pc = Lb % chunks;  // pair chunk
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  int a = 0, b = 0;
  if (npair == NPAIR) {
    int rem = pc * EM_WAVES + w;  // pair 0..35
    while (rem >= 8 - a) { rem -= 8 - a; ++a; }
    b = a + rem;
  } else {
    a = b = pc * EM_WAVES + w;
  }
  const int p = pair_index(a, b);
  const int e = eg * 64 + l;
  const double cuu = g.h * 0.125, cue = g.h * g.h * 0.125, cee = g.h * g.h * g.h * 0.125;
  const int64_t stride = (int64_t)8 * ck.NEcpad;
  double K[NBLK];
#pragma unroll
  for (int q = 0; q < NBLK; ++q) K[q] = 0.0;
  for (int gp = 0; gp < 8; ++gp) {
    __syncthreads();
    {
      // direct global -> LDS loads (no registers involved): each wavefront
      // instruction moves two Hessian components of the group's 64 elements,
      // lanes 0-31 component c and lanes 32-63 component c + 1, 16 B (two
      // elements) per lane, landing at LDS base + 16 * lane
      const double* src = qp + (int64_t)(QP_GRAD + 2 * w + (l >> 5)) * stride + (int64_t)gp * ck.NEcpad + eg * 64 +
                          2 * (l & 31);
#pragma unroll
      for (int r = 0; r < NHP_PAD / (2 * EM_WAVES); ++r) {
        const int c = 2 * (w + EM_WAVES * r);
        __builtin_amdgcn_global_load_lds((const void*)(src + (int64_t)(2 * EM_WAVES * r) * stride),
                                         (__attribute__((address_space(3))) void*)(Ds + c * 64), 16, 0, 0);
      }
      __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    const Shape sa = shape(gp, a), sb = shape(gp, b);
#define DV(pq) Ds[(pq) * 64 + l]
    // u-u: K[i3][k3] += h/8 sum_jl dNa_j dNb_l D(3 i3 + j, 3 k3 + l)
#pragma unroll
    for (int i3 = 0; i3 < 3; ++i3)
#pragma unroll
      for (int k3 = 0; k3 < 3; ++k3) {
        double sacc = 0.0;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
          for (int ll = 0; ll < 3; ++ll) {
            const int pp = 3 * i3 + jj, rr = 3 * k3 + ll;
            const int pq = pp <= rr ? hidx(pp, rr) : hidx(rr, pp);
            sacc += sa.dN[jj] * sb.dN[ll] * DV(pq);
          }
        K[NDOF * i3 + k3] += cuu * sacc;
      }
    // u-eta and eta-u
#pragma unroll
    for (int m = 0; m < NV; ++m)
#pragma unroll
      for (int i3 = 0; i3 < 3; ++i3) {
        const double d0 = DV(hidx(3 * i3, 9 + m)), d1 = DV(hidx(3 * i3 + 1, 9 + m)), d2 = DV(hidx(3 * i3 + 2, 9 + m));
        K[NDOF * i3 + 3 + m] += cue * sb.N * (sa.dN[0] * d0 + sa.dN[1] * d1 + sa.dN[2] * d2);
        K[NDOF * (3 + m) + i3] += cue * sa.N * (sb.dN[0] * d0 + sb.dN[1] * d1 + sb.dN[2] * d2);
      }
    // eta-eta
    const double nn = cee * sa.N * sb.N;
#pragma unroll
    for (int m = 0; m < NV; ++m)
#pragma unroll
      for (int m2 = 0; m2 < NV; ++m2) {
        const int pq = m <= m2 ? hidx(9 + m, 9 + m2) : hidx(9 + m2, 9 + m);
        K[NDOF * (3 + m) + 3 + m2] += nn * DV(pq);
      }
#undef DV
  }
  // gradient energy: h * Lap_ab * Mg (exact under 2x2x2 Gauss)
  const double lap = g.h * lap_ref(a, b);
#pragma unroll
  for (int m = 0; m < NV; ++m)
#pragma unroll
    for (int m2 = 0; m2 < NV; ++m2) K[NDOF * (3 + m) + 3 + m2] += lap * cd->Mg[m][m2];
  if (e < ck.NEc) {
#pragma unroll
    for (int q = 0; q < NBLK; ++q) E[((int64_t)p * NBLK + q) * ck.NEcpad + e] = K[q];
  }
}
__global__ void __launch_bounds__(EM_WAVES * 64, EM_MINB) element_matrix_kernel(Grid g, Chunk ck,
                                                                          const double* __restrict__ qp,
                                                                          const DevCard* __restrict__ cd,
                                                                          double* __restrict__ E, int npair) {
  element_matrix_body(g, ck, qp, cd, E, npair, blockIdx.x, gridDim.x);
}

void launch_element_matrices(const Grid& g, const Chunk& ck, const double* qp, const DevCard* cd, double* elem,
                             hipStream_t s, bool diag_only) {
  const int groups = ck.NEcpad / 64;
  const int npair = diag_only ? 8 : NPAIR;
  const int nb = groups * (npair / EM_WAVES);
  element_matrix_kernel<<<(nb + 7) / 8 * 8, EM_WAVES * 64, 0, s>>>(g, ck, qp, cd, elem, npair);
}

// Stored block (n, n + off(13 + u)) = sum over the <= 8 elements containing
// both nodes of their element blocks, in a fixed order (bitwise reproducible).
// One wavefront per (tile, u): 64 consecutive rows, coalesced element reads
// and coalesced tiled writes.
// nup = NUP: every stored block; nup = 1: the diagonal blocks only.
__device__ __forceinline__ void jacobian_gather_body(const Grid& g, const Chunk& ck, const double* __restrict__ E,
                                                     double* __restrict__ A64, float* __restrict__ A32,
                                                     double* __restrict__ diag64, int nblocks, int nup, int bid,
                                                     int nblk) {
  const int L = xcd_logical(bid, nblk);
  if (L >= nblocks) return;
  const int t = ck.n0 / TILE + L / nup, u = L % nup;
  const int sten = 13 + u;
  const int l = threadIdx.x;
  const int n = t * TILE + l;
  if (n < ck.n0 || n >= ck.n1) return;  // rows of other slabs (no barriers below)
  const int dx = sten % 3 - 1, dy = (sten / 3) % 3 - 1, dz = sten / 9 - 1;
  const bool inside = n < g.N;
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  const int64_t base64 = (int64_t)(t * NUP + u) * Lay<double>::SLICE;
  const int64_t base32 = (int64_t)(t * NUP + u) * Lay<float>::SLICE;
  const int64_t db = (int64_t)t * Lay<double>::SLICE;
  // chunks of three block rows keep 3 NDOF accumulators live
  for (int r0 = 0; r0 < NDOF; r0 += 3) {
    double K[3 * NDOF];
#pragma unroll
    for (int q = 0; q < 3 * NDOF; ++q) K[q] = 0.0;
    if (inside) {
      for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
        const int bx = ax + dx, by = ay + dy, bz = az + dz;
        if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;  // wave-uniform
        const int ex = i - ax, ey = j - ay, ez = k - az;
        if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
        const int b = bx + 2 * by + 4 * bz;
        const int64_t e = ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez) - ck.e0;  // local, in [0, NEc)
        const int64_t es = ck.NEcpad;
        if (a <= b) {
          const double* src = E + (int64_t)pair_index(a, b) * NBLK * es + e;
#pragma unroll
          for (int q = 0; q < 3 * NDOF; ++q) K[q] += src[(int64_t)(NDOF * r0 + q) * es];
        } else {
          const double* src = E + (int64_t)pair_index(b, a) * NBLK * es + e;
#pragma unroll
          for (int rr = 0; rr < 3; ++rr)
#pragma unroll
            for (int c = 0; c < NDOF; ++c) K[NDOF * rr + c] += src[(int64_t)(NDOF * c + r0 + rr) * es];
        }
      }
    }
    if (A64) {
#pragma unroll
      for (int q = 0; q < 3 * NDOF; ++q) A64[base64 + Lay<double>::off(NDOF * r0 + q, l)] = K[q];
    }
    if (A32) {
#pragma unroll
      for (int q = 0; q < 3 * NDOF; ++q) A32[base32 + Lay<float>::off(NDOF * r0 + q, l)] = (float)K[q];
    }
    if (u == 0 && diag64) {
#pragma unroll
      for (int q = 0; q < 3 * NDOF; ++q) diag64[db + Lay<double>::off(NDOF * r0 + q, l)] = K[q];
    }
  }
}
__global__ void __launch_bounds__(64) jacobian_gather_kernel(Grid g, Chunk ck, const double* __restrict__ E,
                                                             double* __restrict__ A64, float* __restrict__ A32,
                                                             double* __restrict__ diag64, int nblocks, int nup) {
  jacobian_gather_body(g, ck, E, A64, A32, diag64, nblocks, nup, blockIdx.x, gridDim.x);
}

void launch_jacobian_gather(const Grid& g, const Chunk& ck, const double* elem, double* A64, float* A32,
                            double* diag64, hipStream_t s, bool diag_only) {
  const int t0 = ck.n0 / TILE, t1 = (ck.n1 + TILE - 1) / TILE;
  const int nup = diag_only ? 1 : NUP;
  const int nblocks = (t1 - t0) * nup;
  const int nb_pad = (nblocks + 7) / 8 * 8;
  jacobian_gather_kernel<<<nb_pad, TILE, 0, s>>>(g, ck, elem, diag_only ? nullptr : A64, diag_only ? nullptr : A32,
                                                 diag64, nblocks, nup);
}

// Symmetric elimination on the stored blocks: entries in constrained rows of
// node n or constrained columns of node m are zeroed, the diagonal of a
// constrained dof is 1.
__device__ __forceinline__ void apply_dirichlet_body(const Grid& g, const uint16_t* __restrict__ mask,
                                                     double* __restrict__ A64, float* __restrict__ A32,
                                                     double* __restrict__ diag64, int nblocks, int bid, int nblk) {
  const int L = xcd_logical(bid, nblk);
  if (L >= nblocks) return;
  const int t = L / NUP, u = L - t * NUP;
  const int sten = 13 + u;
  const int l = threadIdx.x;
  const int n = t * TILE + l;
  if (n >= g.N) return;
  const int dx = sten % 3 - 1, dy = (sten / 3) % 3 - 1, dz = sten / 9 - 1;
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  if (i + dx < 0 || i + dx >= g.nnx || j + dy < 0 || j + dy >= g.nny || k + dz < 0 || k + dz >= g.nnz) return;
  const int m = n + dx + g.nnx * (dy + g.nny * dz);
  const unsigned mr = mask[n], mc = mask[m];
  if ((mr | mc) == 0) return;
  const int64_t base64 = (int64_t)(t * NUP + u) * Lay<double>::SLICE;
  const int64_t base32 = (int64_t)(t * NUP + u) * Lay<float>::SLICE;
  const int64_t db = (int64_t)t * Lay<double>::SLICE;
  for (int e = 0; e < NBLK; ++e) {
    const int r = e / NDOF, c = e % NDOF;
    if (((mr >> r) & 1) || ((mc >> c) & 1)) {
      const double v = (u == 0 && r == c) ? 1.0 : 0.0;
      if (A64) A64[base64 + Lay<double>::off(e, l)] = v;
      if (A32) A32[base32 + Lay<float>::off(e, l)] = (float)v;
      if (u == 0 && diag64) diag64[db + Lay<double>::off(e, l)] = v;
    }
  }
}
__global__ void __launch_bounds__(64) apply_dirichlet_kernel(Grid g, const uint16_t* __restrict__ mask,
                                                             double* __restrict__ A64, float* __restrict__ A32,
                                                             double* __restrict__ diag64, int nblocks) {
  apply_dirichlet_body(g, mask, A64, A32, diag64, nblocks, blockIdx.x, gridDim.x);
}

void launch_apply_dirichlet(const Grid& g, const uint16_t* mask, double* A64, float* A32, double* diag64,
                            hipStream_t s) {
  const int nblocks = g.ntiles * NUP;
  const int nb_pad = (nblocks + 7) / 8 * 8;
  apply_dirichlet_kernel<<<nb_pad, TILE, 0, s>>>(g, mask, A64, A32, diag64, nblocks);
}

// NDOF x NDOF inverse by Gauss-Jordan elimination with partial pivoting (the
// paper's point-block Jacobi inverts each block by LU with partial
// pivoting).  Pivot: the largest magnitude in the column among the rows not
// yet pivoted, ties to the lowest row.
//  * NDOF <= 9: one thread per block, the matrix in registers and inverted in
//    place (Gauss-Jordan on A itself: the pivot row is scaled with the
//    reciprocal on the diagonal, the other rows eliminated with the negated
//    multiples in the pivot column); the row interchanges are selects over
//    the rows below, and are undone as column interchanges in reverse order
//    (the steps invert P A, and A^-1 = (P A)^-1 P), applied as the columns'
//    store positions.
//  * larger blocks: each thread keeps its augmented [A | I] in LDS,
//    lane-interleaved (registers would not hold it).
// DinvS32 (NDOF <= 9; null otherwise): the upper triangle of the FP32
// inverse, packed.  The blocks are symmetric (diagonal blocks of the Hessian
// of the potential, Sec. 3.4), so are their inverses up to rounding.
constexpr bool BI_REGS = NDOF <= 9;
constexpr int BI_THREADS = BI_REGS ? 64 : 16;

__device__ __forceinline__ void block_inverse_regs(const Grid& g, const double* __restrict__ diag64,
                                                   double* __restrict__ Dinv64, float* __restrict__ Dinv32,
                                                   float* __restrict__ DinvS32, int* status, int n) {
  const int t = n / TILE, l = n % TILE;
  const int64_t db = (int64_t)t * Lay<double>::SLICE;
  const int64_t db32 = (int64_t)t * Lay<float>::SLICE;
  const int64_t dbs = (int64_t)t * LaySym<float>::SLICE;
  bool ok = n < g.N;
  double A[NDOF][NDOF];
#pragma unroll
  for (int r = 0; r < NDOF; ++r)
#pragma unroll
    for (int c = 0; c < NDOF; ++c) A[r][c] = ok ? diag64[db + Lay<double>::off(NDOF * r + c, l)] : 0.0;
  int piv[NDOF];
#pragma unroll
  for (int k = 0; k < NDOF; ++k) {
    int p = k;
    double best = fabs(A[k][k]);
#pragma unroll
    for (int r = k + 1; r < NDOF; ++r) {
      const double v = fabs(A[r][k]);
      if (v > best) { best = v; p = r; }
    }
    piv[k] = p;
    ok = ok && best > 0.0;
#pragma unroll
    for (int r = k + 1; r < NDOF; ++r) {
      const bool sw = p == r;
#pragma unroll
      for (int c = 0; c < NDOF; ++c) {
        const double a = A[k][c], b = A[r][c];
        A[k][c] = sw ? b : a;
        A[r][c] = sw ? a : b;
      }
    }
    const double ip = 1.0 / (ok ? A[k][k] : 1.0);
#pragma unroll
    for (int c = 0; c < NDOF; ++c) A[k][c] = (c == k) ? ip : A[k][c] * ip;
#pragma unroll
    for (int r = 0; r < NDOF; ++r) {
      if (r == k) continue;
      const double f = A[r][k];
#pragma unroll
      for (int c = 0; c < NDOF; ++c) A[r][c] = (c == k) ? -f * ip : A[r][c] - f * A[k][c];
    }
  }
  // column interchanges k <-> piv[k] in reverse order, applied through the
  // store: column m of the registers goes to column dst[m] of the inverse
  int dst[NDOF];
#pragma unroll
  for (int m = 0; m < NDOF; ++m) dst[m] = m;
#pragma unroll
  for (int k = NDOF - 1; k >= 0; --k) {
    const int p = piv[k];
#pragma unroll
    for (int m = 0; m < NDOF; ++m) dst[m] = dst[m] == k ? p : (dst[m] == p ? k : dst[m]);
  }
  if (n < g.N && !ok) atomicOr(status, 1);
#pragma unroll
  for (int r = 0; r < NDOF; ++r)
#pragma unroll
    for (int m = 0; m < NDOF; ++m) {
      const double v = ok ? A[r][m] : 0.0;
      if (Dinv64) Dinv64[db + Lay<double>::off(NDOF * r + dst[m], l)] = v;
      if (Dinv32) Dinv32[db32 + Lay<float>::off(NDOF * r + dst[m], l)] = (float)v;
      if (DinvS32 && r <= dst[m]) DinvS32[dbs + LaySym<float>::off(sym_index(r, dst[m]), l)] = (float)v;
    }
}

__device__ __forceinline__ void block_inverse_lds(const Grid& g, const double* __restrict__ diag64,
                                                  double* __restrict__ Dinv64, float* __restrict__ Dinv32,
                                                  int* status, int n) {
  __shared__ double M[NDOF * 2 * NDOF * BI_THREADS];
  const int t = n / TILE, l = n % TILE, lt = threadIdx.x;
  const int64_t db = (int64_t)t * Lay<double>::SLICE;
  const int64_t db32 = (int64_t)t * Lay<float>::SLICE;
#define MM(r, c) M[((r) * 2 * NDOF + (c)) * BI_THREADS + lt]
  bool ok = n < g.N;
  if (ok) {
    for (int r = 0; r < NDOF; ++r)
      for (int c = 0; c < NDOF; ++c) {
        MM(r, c) = diag64[db + Lay<double>::off(NDOF * r + c, l)];
        MM(r, NDOF + c) = (r == c) ? 1.0 : 0.0;
      }
    for (int c = 0; c < NDOF; ++c) {
      int p = c;
      double best = fabs(MM(c, c));
      for (int r = c + 1; r < NDOF; ++r) {
        const double v = fabs(MM(r, c));
        if (v > best) { best = v; p = r; }
      }
      if (!(best > 0.0)) { ok = false; break; }
      if (p != c)
        for (int cc = 0; cc < 2 * NDOF; ++cc) {
          const double tmp = MM(c, cc);
          MM(c, cc) = MM(p, cc);
          MM(p, cc) = tmp;
        }
      const double ip = 1.0 / MM(c, c);
      for (int cc = 0; cc < 2 * NDOF; ++cc) MM(c, cc) *= ip;
      for (int r = 0; r < NDOF; ++r) {
        if (r == c) continue;
        const double f = MM(r, c);
        if (f != 0.0)
          for (int cc = 0; cc < 2 * NDOF; ++cc) MM(r, cc) -= f * MM(c, cc);
      }
    }
    if (!ok) atomicOr(status, 1);
  }
  for (int e = 0; e < NBLK; ++e) {
    const double v = ok ? MM(e / NDOF, NDOF + e % NDOF) : 0.0;
    if (Dinv64) Dinv64[db + Lay<double>::off(e, l)] = v;
    if (Dinv32) Dinv32[db32 + Lay<float>::off(e, l)] = (float)v;
  }
#undef MM
}

__device__ __forceinline__ void block_inverse_body(const Grid& g, const double* __restrict__ diag64,
                                                   double* __restrict__ Dinv64, float* __restrict__ Dinv32,
                                                   float* __restrict__ DinvS32, int* status, int bid) {
  const int n = bid * BI_THREADS + threadIdx.x;
  if (n >= g.Npad) return;
  if constexpr (BI_REGS)
    block_inverse_regs(g, diag64, Dinv64, Dinv32, DinvS32, status, n);
  else
    block_inverse_lds(g, diag64, Dinv64, Dinv32, status, n);
}
__global__ void __launch_bounds__(BI_THREADS) block_inverse_kernel(Grid g, const double* __restrict__ diag64,
                                                                   double* __restrict__ Dinv64,
                                                                   float* __restrict__ Dinv32,
                                                                   float* __restrict__ DinvS32, int* status) {
  block_inverse_body(g, diag64, Dinv64, Dinv32, DinvS32, status, blockIdx.x);
}

void launch_block_inverse(const Grid& g, const double* diag64, double* Dinv64, float* Dinv32, float* DinvS32,
                          int* status, hipStream_t s) {
  block_inverse_kernel<<<(g.Npad + BI_THREADS - 1) / BI_THREADS, BI_THREADS, 0, s>>>(
      g, diag64, Dinv64, Dinv32, BI_REGS ? DinvS32 : nullptr, status);
}

// ---- batched assembly (jobs of many problems in one launch) --------------------
template <int PD, int MIX>
__global__ void __launch_bounds__(128) qp_hess_batch(const AJob* __restrict__ jobs, int njobs) {
  int bid;
  const AJob& j = find_job(jobs, njobs, bid);
  qp_body<true, PD, MIX>(j.g, j.ck, j.state, j.cd, j.qp, bid);
}
__global__ void __launch_bounds__(EM_WAVES * 64, EM_MINB) element_matrix_batch(const AJob* __restrict__ jobs, int njobs) {
  int bid;
  const AJob& j = find_job(jobs, njobs, bid);
  element_matrix_body(j.g, j.ck, j.qp, j.cd, j.elem, j.npair, bid, j.nblk);
}
__global__ void __launch_bounds__(64) jacobian_gather_batch(const AJob* __restrict__ jobs, int njobs) {
  int bid;
  const AJob& j = find_job(jobs, njobs, bid);
  jacobian_gather_body(j.g, j.ck, j.elem, j.A64, j.A32, j.diag64, j.nblocks, j.nup, bid, j.nblk);
}
__global__ void __launch_bounds__(64) apply_dirichlet_batch(const AJob* __restrict__ jobs, int njobs) {
  int bid;
  const AJob& j = find_job(jobs, njobs, bid);
  apply_dirichlet_body(j.g, j.mask, j.A64, j.A32, j.diag64, j.nblocks, bid, j.nblk);
}
__global__ void __launch_bounds__(BI_THREADS) block_inverse_batch(const AJob* __restrict__ jobs, int njobs) {
  int bid;
  const AJob& j = find_job(jobs, njobs, bid);
  block_inverse_body(j.g, j.diag64, j.Dinv64, j.Dinv32, BI_REGS ? j.DinvS32 : nullptr, j.status, bid);
}
__global__ void __launch_bounds__(256) residual_gather_batch(const AJob* __restrict__ jobs, int njobs) {
  int bid;
  const AJob& j = find_job(jobs, njobs, bid);
  residual_gather_body(j.g, j.ck, j.state, j.qp, j.cd, j.R, bid);
}

// the launch shapes of the single-problem launchers, per job
int assembly_job_blocks(int op, AJob& j, bool diag_only) {
  const Grid& g = j.g;
  const Chunk& ck = j.ck;
  switch (op) {
    case AOP_QP_HESS: return (int)(((int64_t)8 * ck.NEcpad + 127) / 128);
    case AOP_ELEMENT: {
      j.npair = diag_only ? 8 : NPAIR;
      const int nb = (ck.NEcpad / 64) * (j.npair / EM_WAVES);
      return (nb + 7) / 8 * 8;
    }
    case AOP_GATHER: {
      const int t0 = ck.n0 / TILE, t1 = (ck.n1 + TILE - 1) / TILE;
      j.nup = diag_only ? 1 : NUP;
      j.nblocks = (t1 - t0) * j.nup;
      return (j.nblocks + 7) / 8 * 8;
    }
    case AOP_DIRICHLET:
      j.nblocks = g.ntiles * NUP;
      return (j.nblocks + 7) / 8 * 8;
    case AOP_BLOCK_INVERSE: return (g.Npad + BI_THREADS - 1) / BI_THREADS;
    case AOP_RESIDUAL: return (ck.n1 - ck.n0 + 255) / 256;
    case AOP_MF_PACK: return mf_pack_job_blocks(j);
    default: return 0;
  }
}

void launch_assembly_batch(int op, int pade, const AJob* jobs, int njobs, int blocks, hipStream_t s) {
  if (njobs <= 0 || blocks <= 0) return;
  switch (op) {
    case AOP_QP_HESS: {  // pade = Pade order + QP_LOG_MIX for logarithmic mixing
      const int pd = pade % QP_LOG_MIX;
      if (pade >= QP_LOG_MIX) {
        if (pd == 11)
          qp_hess_batch<11, 1><<<blocks, 128, 0, s>>>(jobs, njobs);
        else if (pd == 33)
          qp_hess_batch<33, 1><<<blocks, 128, 0, s>>>(jobs, njobs);
        else
          qp_hess_batch<22, 1><<<blocks, 128, 0, s>>>(jobs, njobs);
      } else if (pd == 11) {
        qp_hess_batch<11, 0><<<blocks, 128, 0, s>>>(jobs, njobs);
      } else if (pd == 33) {
        qp_hess_batch<33, 0><<<blocks, 128, 0, s>>>(jobs, njobs);
      } else {
        qp_hess_batch<22, 0><<<blocks, 128, 0, s>>>(jobs, njobs);
      }
      break;
    }
    case AOP_ELEMENT: element_matrix_batch<<<blocks, EM_WAVES * 64, 0, s>>>(jobs, njobs); break;
    case AOP_GATHER: jacobian_gather_batch<<<blocks, TILE, 0, s>>>(jobs, njobs); break;
    case AOP_DIRICHLET: apply_dirichlet_batch<<<blocks, TILE, 0, s>>>(jobs, njobs); break;
    case AOP_BLOCK_INVERSE: block_inverse_batch<<<blocks, BI_THREADS, 0, s>>>(jobs, njobs); break;
    case AOP_RESIDUAL: residual_gather_batch<<<blocks, 256, 0, s>>>(jobs, njobs); break;
    case AOP_MF_PACK: launch_mf_pack_batch(jobs, njobs, blocks, s); break;
    default: break;
  }
}

}  // namespace mvpf
