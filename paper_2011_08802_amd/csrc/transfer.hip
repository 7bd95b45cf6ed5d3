// Grid transfers between nested structured levels (Sec. 3.4: prolongation and
// restriction between the rediscretised levels; state for reassembly).
//  * prolongation P: trilinear interpolation; fine node i takes weight 1 from
//    the coincident coarse node, 1/2 from each of the two coarse neighbours of
//    an edge midpoint, and so on (product of 1D weights);
//  * restriction R = P^T;
//  * state injection: coarse node value = fine value at the coincident node.
// Restricted residuals are zeroed on constrained coarse dofs and prolongated
// corrections are not added on constrained fine dofs.
#include "common.h"

namespace mvpf {

template <typename T>
__device__ __forceinline__ void restrict_body(const Grid& f, const Grid& c, const T* __restrict__ rf,
                                              const uint16_t* __restrict__ cmask, T* __restrict__ bc, int bid) {
  const int I = bid * 256 + threadIdx.x;
  if (I >= c.Npad) return;
  T acc[NDOF] = {};
  unsigned msk = 0x1ff;
  if (I < c.N) {
    msk = cmask[I];
    const int ci = I % c.nnx, cj = (I / c.nnx) % c.nny, ck = I / (c.nnx * c.nny);
    const int fi = 2 * ci, fj = 2 * cj, fk = 2 * ck;
    for (int dz = -1; dz <= 1; ++dz) {
      const int z = fk + dz;
      if (z < 0 || z >= f.nnz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int y = fj + dy;
        if (y < 0 || y >= f.nny) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = fi + dx;
          if (x < 0 || x >= f.nnx) continue;
          const T w = (T)((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
          const int m = x + f.nnx * (y + f.nny * z);
#pragma unroll
          for (int q = 0; q < NDOF; ++q) acc[q] += w * rf[(int64_t)q * f.Npad + m];
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NDOF; ++q) bc[(int64_t)q * c.Npad + I] = ((msk >> q) & 1) ? (T)0 : acc[q];
}
template <typename T>
__global__ void __launch_bounds__(256) restrict_kernel(Grid f, Grid c, const T* __restrict__ rf,
                                                       const uint16_t* __restrict__ cmask, T* __restrict__ bc) {
  restrict_body<T>(f, c, rf, cmask, bc, blockIdx.x);
}

template <typename T>
void launch_restrict(const Grid& fine, const Grid& coarse, const T* rf, const uint16_t* cmask, T* bc,
                     hipStream_t s) {
  restrict_kernel<T><<<(coarse.Npad + 255) / 256, 256, 0, s>>>(fine, coarse, rf, cmask, bc);
}
template void launch_restrict<float>(const Grid&, const Grid&, const float*, const uint16_t*, float*, hipStream_t);
template void launch_restrict<double>(const Grid&, const Grid&, const double*, const uint16_t*, double*,
                                      hipStream_t);

template <typename T>
__device__ __forceinline__ void prolong_add_body(const Grid& f, const Grid& c, const T* __restrict__ ec,
                                                 const uint16_t* __restrict__ fmask, T* __restrict__ xf, int bid) {
  const int n = bid * 256 + threadIdx.x;
  if (n >= f.N) return;
  const unsigned msk = fmask[n];
  if (msk == 0x1ff) return;
  const int i = n % f.nnx, j = (n / f.nnx) % f.nny, k = n / (f.nnx * f.nny);
  int px[2], py[2], pz[2];
  int nxp, nyp, nzp;
  T wx, wy, wz;
  if (i & 1) { px[0] = i >> 1; px[1] = (i >> 1) + 1; nxp = 2; wx = (T)0.5; } else { px[0] = i >> 1; nxp = 1; wx = (T)1; }
  if (j & 1) { py[0] = j >> 1; py[1] = (j >> 1) + 1; nyp = 2; wy = (T)0.5; } else { py[0] = j >> 1; nyp = 1; wy = (T)1; }
  if (k & 1) { pz[0] = k >> 1; pz[1] = (k >> 1) + 1; nzp = 2; wz = (T)0.5; } else { pz[0] = k >> 1; nzp = 1; wz = (T)1; }
  const T w = wx * wy * wz;
  T acc[NDOF] = {};
  for (int a = 0; a < nzp; ++a)
    for (int b = 0; b < nyp; ++b)
      for (int d = 0; d < nxp; ++d) {
        const int m = px[d] + c.nnx * (py[b] + c.nny * pz[a]);
#pragma unroll
        for (int q = 0; q < NDOF; ++q) acc[q] += ec[(int64_t)q * c.Npad + m];
      }
#pragma unroll
  for (int q = 0; q < NDOF; ++q)
    if (!((msk >> q) & 1)) xf[(int64_t)q * f.Npad + n] += w * acc[q];
}
template <typename T>
__global__ void __launch_bounds__(256) prolong_add_kernel(Grid f, Grid c, const T* __restrict__ ec,
                                                          const uint16_t* __restrict__ fmask, T* __restrict__ xf) {
  prolong_add_body<T>(f, c, ec, fmask, xf, blockIdx.x);
}

template <typename T>
void launch_prolong_add(const Grid& fine, const Grid& coarse, const T* ec, const uint16_t* fmask, T* xf,
                        hipStream_t s) {
  prolong_add_kernel<T><<<(fine.Npad + 255) / 256, 256, 0, s>>>(fine, coarse, ec, fmask, xf);
}
template void launch_prolong_add<float>(const Grid&, const Grid&, const float*, const uint16_t*, float*, hipStream_t);
template void launch_prolong_add<double>(const Grid&, const Grid&, const double*, const uint16_t*, double*,
                                         hipStream_t);

__global__ void __launch_bounds__(256) inject_kernel(Grid f, Grid c, const double* __restrict__ sf,
                                                     double* __restrict__ sc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= c.Npad) return;
  if (I >= c.N) {
    for (int q = 0; q < NSTATE; ++q) sc[(int64_t)q * c.Npad + I] = 0.0;
    return;
  }
  const int ci = I % c.nnx, cj = (I / c.nnx) % c.nny, ck = I / (c.nnx * c.nny);
  const int m = 2 * ci + f.nnx * (2 * cj + f.nny * 2 * ck);
#pragma unroll
  for (int q = 0; q < NSTATE; ++q) sc[(int64_t)q * c.Npad + I] = sf[(int64_t)q * f.Npad + m];
}

void launch_inject(const Grid& fine, const Grid& coarse, const double* sf, double* sc, hipStream_t s) {
  inject_kernel<<<(coarse.Npad + 255) / 256, 256, 0, s>>>(fine, coarse, sf, sc);
}

__global__ void __launch_bounds__(256) inject_mask_kernel(Grid f, Grid c, const uint16_t* __restrict__ mf,
                                                          uint16_t* __restrict__ mc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= c.Npad) return;
  if (I >= c.N) { mc[I] = 0; return; }
  const int ci = I % c.nnx, cj = (I / c.nnx) % c.nny, ck = I / (c.nnx * c.nny);
  mc[I] = mf[2 * ci + f.nnx * (2 * cj + f.nny * 2 * ck)];
}

void launch_inject_mask(const Grid& fine, const Grid& coarse, const uint16_t* mf, uint16_t* mc, hipStream_t s) {
  inject_mask_kernel<<<(coarse.Npad + 255) / 256, 256, 0, s>>>(fine, coarse, mf, mc);
}

// ---- batched launches: g = fine grid, g2 = coarse grid of every job ---------
template <typename T>
__global__ void __launch_bounds__(256) restrict_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  restrict_body<T>(j.g, j.g2, (const T*)j.x, j.mask, (T*)j.y, bid);
}
template <typename T>
__global__ void __launch_bounds__(256) prolong_add_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  prolong_add_body<T>(j.g, j.g2, (const T*)j.x, j.mask, (T*)j.y, bid);
}
template <typename T>
void launch_transfer_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s) {
  if (op == BOP_RESTRICT)
    restrict_batch<T><<<blocks, 256, 0, s>>>(jobs, njobs);
  else if (op == BOP_PROLONG)
    prolong_add_batch<T><<<blocks, 256, 0, s>>>(jobs, njobs);
}
template void launch_transfer_batch<float>(int, const BJob*, int, int, hipStream_t);
template void launch_transfer_batch<double>(int, const BJob*, int, int, hipStream_t);

}  // namespace mvpf
