// Galerkin coarse operators, an alternative to the rediscretised coarse
// levels of Sec. 3.4 (opts.coarse = MVPF_COARSE_GALERKIN):
//   A_{l+1} = P~^T A_l P~,
// with P the trilinear prolongation of the V-cycle and P~ = P with the rows of
// constrained level-l unknowns set to zero (the V-cycle never adds a
// correction there), followed by the symmetric elimination of the constrained
// level-(l+1) unknowns.  Where the penalty of the order parameters is active
// on a pattern finer than a coarse element (a state the injected coarse state
// cannot represent), the two constructions differ and only this one keeps the
// coarse correction A-orthogonal to the coarse space.
//
// Built element by element on the nested structured levels: parent element E
// of level l+1 has the 8 children s of level l, and
//   K_E = sum_s W~_s^T K_s W~_s,
//   W~_s[(a, c), (A, c)] = w(a, A) * free_l(node of child corner a, c),
// K_s the child's element matrix (its 36 stored node pairs), w(a, A) the
// trilinear weight of parent corner A at child corner a (a tensor product of
// the 1D weights 1, 1/2, 0 at child positions 0, 1, 2 halves of the parent).
// Summing K_E over the parents that share two nodes (jacobian_gather) gives
// P~^T K P~, which equals P~^T A_l P~ because P~ removes every constrained
// row and column.  Level 0's element matrices come from the Gauss-point
// Hessians (element_matrix, contact included), so the whole hierarchy
// inherits the finest tangent exactly.
#include <utility>

#include "common.h"

namespace mvpf {

// 1D weight of parent corner bit A at child-level position p (0, 1, 2)
__host__ __device__ constexpr double gal_w1(int p, int A) {
  return p == 1 ? 0.5 : ((p == 0) == (A == 0) ? 1.0 : 0.0);
}
// weight of parent corner A at corner a of child s
__host__ __device__ constexpr double gal_w(int s, int a, int A) {
  return gal_w1((s & 1) + (a & 1), A & 1) * gal_w1(((s >> 1) & 1) + ((a >> 1) & 1), (A >> 1) & 1) *
         gal_w1((s >> 2) + (a >> 2), A >> 2);
}
// index of corner a of child s among the parent's 3 x 3 x 3 child-level nodes
__host__ __device__ constexpr int gal_node(int s, int a) {
  return ((s & 1) + (a & 1)) + 3 * (((s >> 1) & 1) + ((a >> 1) & 1)) + 9 * ((s >> 2) + (a >> 2));
}

// acc[pair(A, B)] += w(a, A) w(b, B) k for parent pair I = 8 A + B, A <= B;
// the weights are compile-time constants, zero terms are not generated
template <int S, int a, int b, int I>
__device__ __forceinline__ void gal_term(double k, double (&acc)[NPAIR]) {
  constexpr int A = I >> 3, B = I & 7;
  if constexpr (A <= B) {
    constexpr double w = gal_w(S, a, A) * gal_w(S, b, B);
    if constexpr (w != 0.0) acc[pair_index(A, B)] += w * k;
  }
}
template <int S, int a, int b, int... I>
__device__ __forceinline__ void gal_terms(double k, double (&acc)[NPAIR], std::integer_sequence<int, I...>) {
  (gal_term<S, a, b, I>(k, acc), ...);
}
// the ordered child corner pair (a, b) contributes entry (c, c2) of K_ab to
// entry (c, c2) of the parent blocks, zero where dof c of corner a or dof c2
// of corner b is constrained (fa, fb: free bits of dofs c and c2)
template <int S, int a, int b>
__device__ __forceinline__ void gal_add(double k, uint32_t fa, uint32_t fb, double (&acc)[NPAIR]) {
  const bool keep = ((fa >> gal_node(S, a)) & (fb >> gal_node(S, b)) & 1u) != 0u;
  gal_terms<S, a, b>(keep ? k : 0.0, acc, std::make_integer_sequence<int, 64>{});
}
// stored child pair P (a <= b): its entries q = (c, c2) and qt = (c2, c),
// i.e. K_ab[c][c2] and K_ab[c2][c], are also K_ba[c2][c] and K_ba[c][c2];
// the lane accumulates entry q (accq) and, off the diagonal of the blocks,
// entry qt (acct) of the parent pairs, so each child entry is read once
template <int S, bool DIAG, int P>
__device__ __forceinline__ void gal_child_pair(const double* __restrict__ Ee, int64_t es, int q, int qt, uint32_t fc,
                                               uint32_t fc2, double (&accq)[NPAIR], double (&acct)[NPAIR]) {
  constexpr int a = pair_a(P), b = pair_b(P);
  const double kq = Ee[((int64_t)P * NBLK + q) * es];
  if constexpr (DIAG) {  // c == c2: K_ab[c][c] = K_ba[c][c]
    gal_add<S, a, b>(kq, fc, fc, accq);
    if constexpr (a != b) gal_add<S, b, a>(kq, fc, fc, accq);
  } else {
    const double kt = Ee[((int64_t)P * NBLK + qt) * es];
    gal_add<S, a, b>(kq, fc, fc2, accq);   // K_ab[c][c2]
    gal_add<S, a, b>(kt, fc2, fc, acct);   // K_ab[c2][c]
    if constexpr (a != b) {
      gal_add<S, b, a>(kt, fc, fc2, accq);  // K_ba[c][c2] = K_ab[c2][c]
      gal_add<S, b, a>(kq, fc2, fc, acct);  // K_ba[c2][c] = K_ab[c][c2]
    }
  }
}
template <int S, bool DIAG, int... P>
__device__ __forceinline__ void gal_child(const double* __restrict__ Ee, int64_t es, int q, int qt, uint32_t fc,
                                          uint32_t fc2, double (&accq)[NPAIR], double (&acct)[NPAIR],
                                          std::integer_sequence<int, P...>) {
  (gal_child_pair<S, DIAG, P>(Ee, es, q, qt, fc, fc2, accq, acct), ...);
}

// Block entries handled together: the diagonal ones (c, c) alone, the others
// as the pairs (c, c2), (c2, c) with c < c2: NDOF (NDOF + 1) / 2 tasks.
constexpr int GAL_TASKS = NDOF * (NDOF + 1) / 2;
__device__ __forceinline__ void gal_task(int task, int& c, int& c2) {
  c = 0;
  while (task >= NDOF - c) { task -= NDOF - c; ++c; }
  c2 = c + task;
}

template <bool DIAG>
__device__ __forceinline__ void gal_parent(const Grid& gc, const Chunk& ckc, const double* __restrict__ Ec,
                                           const Grid& gp, int64_t E, int c, int c2, uint32_t fc, uint32_t fc2,
                                           double* __restrict__ Ep) {
  const int q = NDOF * c + c2, qt = NDOF * c2 + c;
  const int X = (int)(E % gp.nx), Y = (int)((E / gp.nx) % gp.ny), Z = (int)(E / ((int64_t)gp.nx * gp.ny));
  double accq[NPAIR], acct[NPAIR];
#pragma unroll
  for (int p = 0; p < NPAIR; ++p) accq[p] = acct[p] = 0.0;
  const int64_t es = ckc.NEcpad;
  const int64_t nxc = gc.nx, nxyc = (int64_t)gc.nx * gc.ny;
  const int64_t e00 = 2 * X + nxc * 2 * Y + nxyc * 2 * Z - ckc.e0;  // child 0, chunk-local
  const std::make_integer_sequence<int, NPAIR> pairs{};
  gal_child<0, DIAG>(Ec + e00, es, q, qt, fc, fc2, accq, acct, pairs);
  gal_child<1, DIAG>(Ec + e00 + 1, es, q, qt, fc, fc2, accq, acct, pairs);
  gal_child<2, DIAG>(Ec + e00 + nxc, es, q, qt, fc, fc2, accq, acct, pairs);
  gal_child<3, DIAG>(Ec + e00 + nxc + 1, es, q, qt, fc, fc2, accq, acct, pairs);
  gal_child<4, DIAG>(Ec + e00 + nxyc, es, q, qt, fc, fc2, accq, acct, pairs);
  gal_child<5, DIAG>(Ec + e00 + nxyc + 1, es, q, qt, fc, fc2, accq, acct, pairs);
  gal_child<6, DIAG>(Ec + e00 + nxyc + nxc, es, q, qt, fc, fc2, accq, acct, pairs);
  gal_child<7, DIAG>(Ec + e00 + nxyc + nxc + 1, es, q, qt, fc, fc2, accq, acct, pairs);
#pragma unroll
  for (int p = 0; p < NPAIR; ++p) Ep[((int64_t)p * NBLK + q) * gp.NEpad + E] = accq[p];
  if constexpr (!DIAG) {
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) Ep[((int64_t)p * NBLK + qt) * gp.NEpad + E] = acct[p];
  }
}

// One wavefront per 64 consecutive parents and one task: block entry (c, c)
// or the entry pair (c, c2), (c2, c).  Each lane accumulates those entries of
// its parent's 36 node pairs over the 8 children and their corner pairs, in
// a fixed order (bitwise reproducible), reading each child entry it needs
// once.  The tasks of one parent group are consecutive logical workgroups on
// one XCD.  Child element matrices: chunk-local, Ec[(p NBLK + q) es + e - e0];
// parents: whole level, Ep[(P NBLK + q) NEpad + E], E in [E0, E1).
__global__ void __launch_bounds__(64) galerkin_coarsen_kernel(Grid gc, Chunk ckc, const double* __restrict__ Ec,
                                                             const uint16_t* __restrict__ maskc, Grid gp,
                                                             int64_t E0, int64_t E1, int nwork, double* __restrict__ Ep) {
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nwork) return;
  int c, c2;
  gal_task(L % GAL_TASKS, c, c2);
  const int64_t E = E0 + (int64_t)(L / GAL_TASKS) * 64 + threadIdx.x;
  if (E >= E1) return;
  const int X = (int)(E % gp.nx), Y = (int)((E / gp.nx) % gp.ny), Z = (int)(E / ((int64_t)gp.nx * gp.ny));
  // free bits of dofs c (fc) and c2 (fc2) of the parent's 27 child-level nodes
  uint32_t fc = 0, fc2 = 0;
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    const int64_t node = (2 * X + k % 3) + (int64_t)gc.nnx * ((2 * Y + (k / 3) % 3) + (int64_t)gc.nny * (2 * Z + k / 9));
    const uint32_t m = maskc[node];
    fc |= ((~m >> c) & 1u) << k;
    fc2 |= ((~m >> c2) & 1u) << k;
  }
  if (c == c2)
    gal_parent<true>(gc, ckc, Ec, gp, E, c, c2, fc, fc2, Ep);
  else
    gal_parent<false>(gc, ckc, Ec, gp, E, c, c2, fc, fc2, Ep);
}

void launch_galerkin_coarsen(const Grid& gc, const Chunk& ckc, const double* Ec, const uint16_t* maskc,
                             const Grid& gp, int Z0, int Z1, double* Ep, hipStream_t s) {
  const int64_t nxy = (int64_t)gp.nx * gp.ny;
  const int64_t E0 = Z0 * nxy, E1 = Z1 * nxy;
  if (E1 <= E0) return;
  const int64_t nwork = (E1 - E0 + 63) / 64 * GAL_TASKS;
  const int blocks = (int)((nwork + 7) / 8 * 8);
  galerkin_coarsen_kernel<<<blocks, 64, 0, s>>>(gc, ckc, Ec, maskc, gp, E0, E1, (int)nwork, Ep);
}

}  // namespace mvpf
