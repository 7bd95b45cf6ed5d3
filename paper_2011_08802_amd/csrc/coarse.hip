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

// one thread per (node, stored block, block row): the NDOF entries of that row
// and, for off-diagonal blocks, their transposes (the lower half)
__global__ void __launch_bounds__(256) dense_from_bsr_kernel(Grid g, const double* __restrict__ A,
                                                             double* __restrict__ D) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.N * NUP * NDOF) return;
  const int r = idx % NDOF, u = (idx / NDOF) % NUP, n = idx / (NDOF * NUP);
  const int64_t nd = (int64_t)NDOF * g.N;
  const int t = n >> 6, l = n & 63;
  const int i = n % g.nnx, j = (n / g.nnx) % g.nny, k = n / (g.nnx * g.nny);
  const int s = 13 + u;
  const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
  if (i + dx < 0 || i + dx >= g.nnx || j + dy < 0 || j + dy >= g.nny || k + dz < 0 || k + dz >= g.nnz) return;
  const int m = n + dx + g.nnx * (dy + g.nny * dz);
  const double* Ab = A + (int64_t)(t * NUP + u) * Lay<double>::SLICE;
#pragma unroll
  for (int c = 0; c < NDOF; ++c) {
    const double v = Ab[Lay<double>::off(r * NDOF + c, l)];
    D[((int64_t)r * g.N + n) * nd + (int64_t)c * g.N + m] = v;
    if (u > 0) D[((int64_t)c * g.N + m) * nd + (int64_t)r * g.N + n] = v;  // lower half by symmetry
  }
}

__global__ void zero_kernel_d(int64_t n, double* p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

void launch_dense_from_bsr(const Grid& g, const double* A64, double* dense, hipStream_t s) {
  const int64_t nd = (int64_t)NDOF * g.N;
  zero_kernel_d<<<1024, 256, 0, s>>>(nd * nd, dense);
  dense_from_bsr_kernel<<<(g.N * NUP * NDOF + 255) / 256, 256, 0, s>>>(g, A64, dense);
}

// Two-level blocked Gauss-Jordan inversion with partial pivoting.
//
// M = [A | Y] is n x 2n, row-major.  Y starts at zero; the k-th pivot row
// p_k (the row chosen for column k) gets its unit vector e_{p_k} placed in
// column n + k at the moment it is chosen, so the right half ends up holding
// T e_{p_k}, where T is the product of all elimination steps.  Since
// T A = E with E[p_k][k] = 1, row k of A^-1 is row p_k of T, i.e.
// A^-1[k][p_m] = M[p_k][n + m].
//
// Outer panels of NB columns c0 .. c0 + nbw - 1.  Inside a panel, sub-panels
// of PB columns are eliminated with partial pivoting by
//   0. gj_fetch: copies the sub-panel F = M[:, sub-panel] (row-major F and
//      column-major Wc);
//   1. gj_panel: one workgroup holds the sub-panel in registers, chooses the
//      pivot rows by elimination with partial pivoting restricted to the
//      sub-panel (rows pivoted earlier are excluded), places the unit
//      columns and inverts the pivot block Mp = F[P, :] (Gauss-Jordan in
//      LDS, rows in pivot order); beyond 4 GJ_THREADS rows the same is done
//      by tournament pivoting (gj_tourn0, gj_tourn1);
//   2. gj_rows: R = Mp^-1 M[P, active] (the new pivot rows);
//   3. gj_update: rows in P become R, every other row i becomes
//      M[i, active] - F[i, :] R,
// where "active" is only the outer panel's 2 nbw columns [c0, c0 + nbw) and
// [n + c0, n + c0 + nbw).  Columns outside the active set are either
// untouched by these steps (eliminated unit columns, zero columns of Y) or
// are updated once per outer panel: with T_o the panel's accumulated
// transformation, T_o - I is non-zero only in the columns p_k, whose values
// T_o e_{p_k} - e_{p_k} =: Yo[:, k] sit in the right half, so
//   M[:, rest] += Yo * M_old[P, rest],   rest = [c0 + nbw, n + c0)
// (gj_gather copies Yo and the old pivot rows; gj_gemm does the product).
constexpr int GJB = 32;   // widest sub-panel
constexpr int GJ_NB = 128;  // outer panel width
constexpr int GJ_THREADS = 512;

// Several inversions can run as one: every kernel below takes a job table
// (workgroup z of a launch works on job sel[z], or z without a selection
// list) or, for a single inversion, the job by value.  Each job keeps its
// own sub-panel width and kernel variant, so a job computes the same
// numbers alone or in a batch.
struct GJJobs {
  const GJJob* tab;  // device table, or nullptr: use the job passed by value
  const int* sel;    // device selection list (job indices), or nullptr
};
__device__ __forceinline__ const GJJob& gj_job(const GJJobs& J, const GJJob& one) {
  if (!J.tab) return one;
  return J.tab[J.sel ? J.sel[blockIdx.z] : blockIdx.z];
}
// sub-panel width: up to 4 rows per thread the sub-panel is factored in one
// workgroup's registers, beyond that by tournament pivoting
__host__ __device__ inline int gj_pbw(int n) { return (n > 4 * GJ_THREADS || n <= 2 * GJ_THREADS) ? GJB : 16; }
// the job's sub-panel at (c0, s0), if it has one: outer-panel width nbw, width B
__device__ __forceinline__ bool gj_step(int n, int c0, int s0, int& nbw, int& B) {
  if (c0 >= n) return false;
  nbw = min(GJ_NB, n - c0);
  const int pb = gj_pbw(n);
  if (s0 >= c0 + nbw || (s0 - c0) % pb) return false;
  B = min(pb, c0 + nbw - s0);
  return true;
}

// Inverse of the pivot block Mp = F[pr[a], b] (B x B, B <= PB), rows in
// pivot order, by Gauss-Jordan on [Mp | I] in LDS.  No pivot search: each
// pivot was the largest remaining entry of its column over all candidate
// rows, these rows included, so in pivot order the diagonal is the
// partial-pivoting choice.  Needs blockDim.x >= 2 B; 2 barriers per column.
template <int PB>
__device__ void pivot_block_inverse(int B, const double* __restrict__ F, const int* pr, double* __restrict__ Pinv,
                                    int* status, double (*Mp)[2 * PB], double* fr, double* rowc) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < B * B; idx += blockDim.x) {
    const int a = idx / B, b = idx % B;
    Mp[a][b] = F[(int64_t)pr[a] * B + b];
    Mp[a][B + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < B; ++c) {
    const double piv = Mp[c][c];
    if (!(fabs(piv) > 0.0)) {
      if (tid == 0) atomicOr(status, 1);
      return;  // uniform
    }
    if (tid < 2 * B) rowc[tid] = Mp[c][tid] / piv;
    if (tid < B) fr[tid] = Mp[tid][c];
    __syncthreads();
    for (int idx = tid; idx < B * 2 * B; idx += blockDim.x) {
      const int r = idx / (2 * B), cc = idx % (2 * B);
      Mp[r][cc] = (r == c) ? rowc[cc] : Mp[r][cc] - fr[r] * rowc[cc];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < B * B; idx += blockDim.x) Pinv[idx] = Mp[idx / B][B + idx % B];
}

// Elimination with partial pivoting over the rows a workgroup holds in its
// registers: W[q][.] is the sub-panel window of row rid[q] (act[q]: still a
// candidate).  After each step the windows shift left by one, so the active
// column is always W[q][0] (all register indices static).  One barrier per
// column: every wavefront's best row publishes its value, index and window
// in LDS slots (double-buffered by column parity), and every wavefront picks
// the block's winner from the slots itself; ties go to the lowest row.
// Candidates are ordered by |entry|, then by the lower row; the order is
// total, so the winner does not depend on the order in which pairs are
// compared.  Inside a wavefront the comparisons run over DPP lane exchanges
// and scalar lane reads (no LDS round trips).
// on_pivot(jj, p) runs in the thread that holds the chosen row p; it writes
// LDS only, since a global store in the loop would hold up the next barrier
// (flat stores count against the LDS wait counter).
// strict: a column without a non-zero candidate makes the block singular
// (returns -1); otherwise such a column takes its lowest candidate row without
// elimination, and the loop ends early (returns the count) when no candidate
// rows are left.
constexpr int NWV = GJ_THREADS / 64;
static_assert(NWV == 8, "the slot reduction covers one group of 8 lanes");

// (ov, oi) beats (v, idx): a candidate (row >= 0) beats none, then the larger
// value, then the lower row
__device__ __forceinline__ bool cand_better(double ov, int oi, double v, int idx) {
  return oi >= 0 && (idx < 0 || ov > v || (ov == v && oi < idx));
}
template <int CTRL>
__device__ __forceinline__ void cand_step(double& v, int& idx, int& slot) {
  const double ov = dpp_t<CTRL>(v);
  const int oi = dpp_i<CTRL>(idx), os = dpp_i<CTRL>(slot);
  if (cand_better(ov, oi, v, idx)) { v = ov; idx = oi; slot = os; }
}
// the best of groups of 8 lanes in each of their lanes: xor 1, xor 2, then the
// half-row mirror (lane i <-> 7 - i) joins the two quads
__device__ __forceinline__ void cand_best8(double& v, int& idx, int& slot) {
  cand_step<0xB1>(v, idx, slot);
  cand_step<0x4E>(v, idx, slot);
  cand_step<0x141>(v, idx, slot);
}
// the best of lane `src` of the wavefront, in every lane
__device__ __forceinline__ void cand_read(double& v, int& idx, int& slot, int src) {
  v = read_lane(v, src);
  idx = __builtin_amdgcn_readlane(idx, src);
  slot = __builtin_amdgcn_readlane(slot, src);
}
// the best of the wavefront in every lane: rows of 16 lanes by DPP (groups of
// 8, then the row mirror lane i <-> 15 - i), then the four rows from scalar
// reads of lanes 0, 16, 32 and 48
__device__ __forceinline__ void cand_best64(double& v, int& idx, int& slot) {
  cand_best8(v, idx, slot);
  cand_step<0x140>(v, idx, slot);
  double bv = v;
  int bi = idx, bs = slot;
  cand_read(bv, bi, bs, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    double ov = v;
    int oi = idx, os = slot;
    cand_read(ov, oi, os, r);
    if (cand_better(ov, oi, bv, bi)) { bv = ov; bi = oi; bs = os; }
  }
  v = bv;
  idx = bi;
  slot = bs;
}

// NW: wavefronts of the workgroup (at most NWV)
template <int RPT, int PB, int NW, typename OnPivot>
__device__ int window_eliminate(double (&W)[RPT][PB], bool (&act)[RPT], const int (&rid)[RPT], int B, bool strict,
                                OnPivot on_pivot, double (*cv)[NWV], int (*ci)[NWV], double (*crow)[NWV][PB]) {
  static_assert(NW >= 1 && NW <= NWV, "one slot per wavefront");
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
#pragma unroll 1
  for (int jj = 0; jj < B; ++jj) {
    double v = -1.0;
    int idx = -1;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const double cand = fabs(W[q][0]);
      if (act[q] && (cand > v || (cand == v && rid[q] < idx))) { v = cand; idx = rid[q]; }
    }
    int unused = 0;
    cand_best64(v, idx, unused);
    const int par = jj & 1;
    bool mine = false;
#pragma unroll
    for (int q = 0; q < RPT; ++q) mine = mine || (act[q] && rid[q] == idx);
    if (lane == 0) {
      cv[par][wid] = v;
      ci[par][wid] = idx;
    }
    if (idx >= 0 && mine) {
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (act[q] && rid[q] == idx) {
#pragma unroll
          for (int b = 0; b < PB; ++b) crow[par][wid][b] = W[q][b];
        }
    }
    __syncthreads();
    // lanes 0 .. NW - 1 take one slot each; the best of them, in every lane
    double bv = -1.0;
    int p = -1, pw = 0;
    if (lane < NW) {
      bv = cv[par][lane];
      p = ci[par][lane];
      pw = lane;
    }
    cand_best8(bv, p, pw);
    cand_read(bv, p, pw, 0);
    if (p < 0) return strict ? -1 : jj;  // uniform: no candidate rows left
    if (strict && !(bv > 0.0)) return -1;  // uniform: singular
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (act[q] && rid[q] == p) {
        act[q] = false;
        on_pivot(jj, p);
      }
    const double* prw = crow[par][pw];
    const double ip = bv > 0.0 ? 1.0 / prw[0] : 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const double f = act[q] ? W[q][0] * ip : 0.0;
#pragma unroll
      for (int b = 1; b < PB; ++b) W[q][b - 1] = W[q][b] - f * prw[b];
      W[q][PB - 1] = 0.0;
    }
  }
  return B;
}

// Sub-panel factorisation (columns c0 .. c0 + B - 1) in one workgroup of NT
// threads.  Thread t owns rows t, t + NT, ... (RPT of them); n <= NT * RPT.
// A column costs every wavefront the same pivot search whatever its row
// count, so fewer, fuller wavefronts (NT = 256, 5 rows per thread) take less
// time per column than 512 threads with 3 rows each.
template <int RPT, int PB, int NT>
__global__ void __launch_bounds__(NT) gj_panel_kernel(GJJobs J, GJJob one, int oc0, int c0) {
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  int nbw_, B;
  if (!gj_step(n, oc0, c0, nbw_, B)) return;  // uniform
  double* __restrict__ M = jb.M;
  const double* __restrict__ F = jb.F;
  const double* __restrict__ Wc = jb.Wc;
  int* __restrict__ done = jb.done;
  int* __restrict__ prow = jb.prow;
  double* __restrict__ Pinv = jb.Pinv;
  int* status = jb.status;
  __shared__ double Mp[PB][2 * PB];
  __shared__ double fr[PB];
  __shared__ double rowc[2 * PB];
  __shared__ int pr[PB];
  __shared__ double cv[2][NWV];
  __shared__ int ci[2][NWV];
  __shared__ double crow[2][NWV][PB];
  const int tid = threadIdx.x;
  const int64_t w = 2 * (int64_t)n;
  double W[RPT][PB];
  bool act[RPT];
  int rid[RPT];
  // The sub-panel comes column-major from gj_fetch (Wc[b][i], F = its
  // row-major copy), so the loads of a wavefront are 64 consecutive rows.
  // Addresses are clamped and loaded unconditionally (all in flight at
  // once); window entries of rows i >= n or columns b >= B are never used
  // (such rows are inactive, and window positions at or beyond B - jj never
  // become the active column).
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = tid + q * NT;
    const bool ok = i < n;
    const int ic = ok ? i : 0;
    rid[q] = i;
    act[q] = !done[ic] && ok;
#pragma unroll
    for (int b = 0; b < PB; ++b) W[q][b] = Wc[(int64_t)(b < B ? b : B - 1) * n + ic];
  }
  // the pivots go to LDS during the elimination and to global memory after it
  // (a global store inside the column loop would hold up every barrier)
  const int got =
      window_eliminate<RPT, PB, NT / 64>(W, act, rid, B, true, [&](int jj, int p) { pr[jj] = p; }, cv, ci, crow);
  if (got < 0) {
    if (tid == 0) atomicOr(status, 1);
    return;  // uniform
  }
  __syncthreads();  // pr[] complete
  pivot_block_inverse<PB>(B, F, pr, Pinv, status, Mp, fr, rowc);
  if (tid < B) {  // after the inverse's barriers, which would wait for these stores
    const int p = pr[tid];
    done[p] = 1;
    prow[c0 + tid] = p;
    M[(int64_t)p * w + n + c0 + tid] = 1.0;  // unit column of the new pivot
  }
}

// active column j (0 .. 2 nbw - 1) of the outer panel at c0
__device__ __forceinline__ int64_t gj_col(int n, int c0, int nbw, int j) {
  return j < nbw ? (int64_t)c0 + j : (int64_t)n + c0 + (j - nbw);
}

// R[a][j] = sum_b Pinv[a][b] M[prow[s0 + b]][col(j)] over the active columns
__global__ void __launch_bounds__(256) gj_rows_kernel(GJJobs J, GJJob one, int c0, int s0) {
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  int nbw, B;
  if (!gj_step(n, c0, s0, nbw, B)) return;
  const double* __restrict__ M = jb.M;
  const int* __restrict__ prow = jb.prow;
  const double* __restrict__ Pinv = jb.Pinv;
  double* __restrict__ R = jb.R;
  const int64_t w = 2 * (int64_t)n;
  const int a = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= B || j >= 2 * nbw) return;
  const int64_t c = gj_col(n, c0, nbw, j);
  double mv[GJB];
#pragma unroll
  for (int b = 0; b < GJB; ++b) mv[b] = M[(int64_t)prow[s0 + (b < B ? b : B - 1)] * w + c];  // all loads at once
  double s = 0.0;
#pragma unroll
  for (int b = 0; b < GJB; ++b)
    if (b < B) s += Pinv[a * B + b] * mv[b];
  R[(int64_t)a * 2 * nbw + j] = s;
}

// Over the active columns: rows pivoted in this sub-panel become R, every
// other row i becomes M[i] - F[i, :] R.  Block: UPR rows x 256 columns.
constexpr int UPR = 8;
__global__ void __launch_bounds__(256) gj_update_kernel(GJJobs J, GJJob one, int c0, int s0) {
  __shared__ double Fs[UPR][GJB];
  __shared__ int sub[UPR];  // sub-panel position of each row, or -1
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  int nbw, B;
  if (!gj_step(n, c0, s0, nbw, B)) return;  // uniform
  const int r0 = blockIdx.y * UPR;
  if (r0 >= n || blockIdx.x * 256 >= 2 * nbw) return;  // uniform, before the barriers
  double* __restrict__ M = jb.M;
  const double* __restrict__ F = jb.F;
  const double* __restrict__ R = jb.R;
  const int* __restrict__ prow = jb.prow;
  const int64_t w = 2 * (int64_t)n;
  const int j = blockIdx.x * 256 + threadIdx.x;
  for (int idx = threadIdx.x; idx < UPR * GJB; idx += 256) {
    const int rr = idx / GJB, b = idx % GJB;
    Fs[rr][b] = (r0 + rr < n && b < B) ? F[(int64_t)(r0 + rr) * B + b] : 0.0;
  }
  if (threadIdx.x < UPR) sub[threadIdx.x] = -1;
  __syncthreads();
  if (threadIdx.x < B) {
    const int pr = prow[s0 + threadIdx.x];
    if (pr >= r0 && pr < r0 + UPR) sub[pr - r0] = threadIdx.x;
  }
  __syncthreads();
  if (j >= 2 * nbw) return;
  const int64_t c = gj_col(n, c0, nbw, j);
  // unconditional clamped loads; entries b >= B meet zero padding in Fs and
  // are never selected as a pivot row's value
  double Rc[GJB];
#pragma unroll
  for (int b = 0; b < GJB; ++b) Rc[b] = R[(int64_t)(b < B ? b : B - 1) * 2 * nbw + j];
  // all rows' old values are loaded before the first store (each store would
  // otherwise complete before the next row's load is waited for)
  int sr[UPR];
#pragma unroll
  for (int rr = 0; rr < UPR; ++rr) sr[rr] = sub[rr];
  double old[UPR];
#pragma unroll
  for (int rr = 0; rr < UPR; ++rr) {
    const int i = r0 + rr;
    old[rr] = (i < n && sr[rr] < 0) ? M[(int64_t)i * w + c] : 0.0;
  }
#pragma unroll
  for (int rr = 0; rr < UPR; ++rr) {
    const int i = r0 + rr;
    if (i >= n) break;
    const int pi = sr[rr];
    double v;
    if (pi >= 0) {
      v = Rc[0];
#pragma unroll
      for (int b = 1; b < GJB; ++b)
        if (b == pi) v = Rc[b];
    } else {
      v = old[rr];
#pragma unroll
      for (int b = 0; b < GJB; ++b) v -= Fs[rr][b] * Rc[b];
    }
    M[(int64_t)i * w + c] = v;
  }
}

// ---- wide sub-panels (n > 4 GJ_THREADS): tournament pivoting -------------
// Beyond 4 rows per thread a sub-panel (B = GJB columns) no longer fits one
// workgroup's registers.  Its pivot rows are chosen by tournament pivoting
// (communication-avoiding LU, Grigori, Demmel and Xiang 2011) in two rounds:
//   gj_tourn0: each block of GJ_THREADS rows eliminates the sub-panel over its
//              own candidate rows and nominates the rows it pivoted on;
//   gj_tourn1: one workgroup eliminates the original sub-panel rows of all
//              nominees (at most 16 x GJB <= GJ_THREADS of them) and takes its
//              pivots as the sub-panel's, then inverts the pivot block.
// The pivots differ from column-by-column partial pivoting over all rows
// (each is the largest among the nominees); the inverse is the same up to
// rounding.  Two launches per sub-panel instead of one per column.

// F[i][b] = Wc[b][i] = M[i][s0 + b]
__global__ void __launch_bounds__(256) gj_fetch_kernel(GJJobs J, GJJob one, int c0, int s0) {
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  int nbw, B;
  if (!gj_step(n, c0, s0, nbw, B)) return;
  const double* __restrict__ M = jb.M;
  double* __restrict__ F = jb.F;
  double* __restrict__ Wc = jb.Wc;
  const int64_t w = 2 * (int64_t)n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * B) return;
  const int i = (int)(idx / B), b = (int)(idx - (int64_t)i * B);
  const double v = M[(int64_t)i * w + s0 + b];
  F[idx] = v;
  Wc[(int64_t)b * n + i] = v;
}

__global__ void __launch_bounds__(GJ_THREADS) gj_tourn0_kernel(GJJobs J, GJJob one, int c0, int s0) {
  __shared__ double cv[2][NWV];
  __shared__ int ci[2][NWV];
  __shared__ double crow[2][NWV][GJB];
  __shared__ int pv[GJB];  // the block's pivot rows (written to global memory after the elimination)
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  int nbw, B;
  if (!gj_step(n, c0, s0, nbw, B)) return;  // uniform
  if ((int)blockIdx.x * GJ_THREADS >= n) return;  // uniform: beyond the job's row blocks
  const double* __restrict__ Wc = jb.Wc;
  const int* __restrict__ done = jb.done;
  int* __restrict__ cand = jb.cand;
  const int i = blockIdx.x * GJ_THREADS + threadIdx.x;
  const bool ok = i < n;
  const int ic = ok ? i : 0;
  double W[1][GJB];
  bool act[1] = {!done[ic] && ok};
  const int rid[1] = {i};
#pragma unroll
  for (int b = 0; b < GJB; ++b) W[0][b] = Wc[(int64_t)(b < B ? b : B - 1) * n + ic];
  int* mine = cand + blockIdx.x * GJB;
  const int got =
      window_eliminate<1, GJB, NWV>(W, act, rid, B, false, [&](int jj, int p) { pv[jj] = p; }, cv, ci, crow);
  __syncthreads();  // pv[] complete
  for (int jj = threadIdx.x; jj < GJB; jj += blockDim.x) mine[jj] = jj < got ? pv[jj] : -1;
}

__global__ void __launch_bounds__(GJ_THREADS) gj_tourn1_kernel(GJJobs J, GJJob one, int c0, int s0) {
  __shared__ double Mp[GJB][2 * GJB];
  __shared__ double fr[GJB];
  __shared__ double rowc[2 * GJB];
  __shared__ int pr[GJB];
  __shared__ double cv[2][NWV];
  __shared__ int ci[2][NWV];
  __shared__ double crow[2][NWV][GJB];
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  int nbw, B;
  if (!gj_step(n, c0, s0, nbw, B)) return;  // uniform
  const int nblk = (n + GJ_THREADS - 1) / GJ_THREADS;
  double* __restrict__ M = jb.M;
  const double* __restrict__ F = jb.F;
  const int* __restrict__ cand = jb.cand;
  int* __restrict__ done = jb.done;
  int* __restrict__ prow = jb.prow;
  double* __restrict__ Pinv = jb.Pinv;
  int* status = jb.status;
  const int tid = threadIdx.x;
  const int64_t w = 2 * (int64_t)n;
  const int r = tid < nblk * GJB ? cand[tid] : -1;
  const int rc = r >= 0 ? r : 0;
  double W[1][GJB];
  bool act[1] = {r >= 0};
  const int rid[1] = {r >= 0 ? r : n + tid};  // distinct ids for empty slots (never active)
#pragma unroll
  for (int b = 0; b < GJB; ++b) W[0][b] = F[(int64_t)rc * B + (b < B ? b : B - 1)];
  const int got =
      window_eliminate<1, GJB, NWV>(W, act, rid, B, true, [&](int jj, int p) { pr[jj] = p; }, cv, ci, crow);
  if (got < 0) {
    if (tid == 0) atomicOr(status, 1);
    return;  // uniform
  }
  __syncthreads();  // pr[] complete
  pivot_block_inverse<GJB>(B, F, pr, Pinv, status, Mp, fr, rowc);
  if (tid < B) {
    const int p = pr[tid];
    done[p] = 1;
    prow[s0 + tid] = p;
    M[(int64_t)p * w + n + s0 + tid] = 1.0;
  }
}

// Yo[i][k] = M[i][n + c0 + k] - [i == p_{c0+k}];  Rb[k][j] = M[p_{c0+k}][c0 + nbw + j]
__global__ void __launch_bounds__(256) gj_gather_kernel(GJJobs J, GJJob one, int c0) {
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  if (c0 >= n) return;
  const int nbw = min(GJ_NB, n - c0);
  const double* __restrict__ M = jb.M;
  const int* __restrict__ prow = jb.prow;
  double* __restrict__ Yo = jb.Yo;
  double* __restrict__ Rb = jb.Rb;
  const int64_t w = 2 * (int64_t)n;
  const int64_t nr = n - nbw;
  const int64_t ny = (int64_t)n * nbw, nrb = (int64_t)nbw * nr;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ny + nrb;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < ny) {
      const int64_t i = idx / nbw;
      const int k = (int)(idx - i * nbw);
      Yo[idx] = M[i * w + n + c0 + k] - ((int)i == prow[c0 + k] ? 1.0 : 0.0);
    } else {
      const int64_t t = idx - ny;
      const int k = (int)(t / nr);
      const int64_t jj = t - (int64_t)k * nr;
      Rb[t] = M[(int64_t)prow[c0 + k] * w + c0 + nbw + jj];
    }
  }
}

// M[i][c0 + nbw + j] += sum_k Yo[i][k] Rb[k][j]  (i < n, j < n - nbw).
// 64 x 64 output tile per workgroup, 4 x 4 per thread, K staged in LDS by 16.
constexpr int GT = 64, GK = 16;
__global__ void __launch_bounds__(256) gj_gemm_kernel(GJJobs J, GJJob one, int c0) {
  __shared__ double Ys[GK][GT + 1];
  __shared__ double Rs[GK][GT + 1];
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  if (c0 >= n) return;  // uniform
  const int nbw = min(GJ_NB, n - c0);
  const int nr = n - nbw;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  if (i0 >= n || j0 >= nr) return;  // uniform, before the barriers
  const double* __restrict__ Yo = jb.Yo;
  const double* __restrict__ Rb = jb.Rb;
  double* __restrict__ M = jb.M;
  const int64_t w = 2 * (int64_t)n;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < nbw; k0 += GK) {
    for (int idx = threadIdx.x; idx < GK * GT; idx += 256) {
      const int kk = idx % GK, ii = idx / GK;   // Yo: consecutive threads walk k
      const int i = i0 + ii, k = k0 + kk;
      Ys[kk][ii] = (i < n && k < nbw) ? Yo[(int64_t)i * nbw + k] : 0.0;
      const int jj = idx % GT, kr = idx / GT;   // Rb: consecutive threads walk j
      const int jc = j0 + jj, k2 = k0 + kr;
      Rs[kr][jj] = (jc < nr && k2 < nbw) ? Rb[(int64_t)k2 * nr + jc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) { a[q] = Ys[kk][ty + 16 * q]; b[q] = Rs[kk][tx + 16 * q]; }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int i = i0 + ty + 16 * x;
    if (i >= n) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int jc = j0 + tx + 16 * y;
      if (jc < nr) M[(int64_t)i * w + c0 + nbw + jc] += acc[x][y];
    }
  }
}

__global__ void __launch_bounds__(256) gj_init_kernel(GJJobs J, GJJob one) {
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  const double* __restrict__ a = jb.a;
  double* __restrict__ M = jb.M;
  int* __restrict__ done = jb.done;
  int* __restrict__ prow = jb.prow;
  int* __restrict__ cand = jb.cand;
  const int64_t w = 2 * (int64_t)n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * w;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / w, c = idx - i * w;
    M[idx] = (c < n) ? a[i * n + c] : 0.0;
    if (c == 0) {
      done[i] = 0;
      prow[i] = 0;  // any valid row until the pivot is chosen
      if (i < 16 * GJB) cand[i] = -1;
    }
  }
}

// A^-1[k][p_m] = M[p_k][n + m]
__global__ void __launch_bounds__(256) gj_extract_kernel(GJJobs J, GJJob one) {
  const GJJob& jb = gj_job(J, one);
  const int n = jb.n;
  const double* __restrict__ M = jb.M;
  const int* __restrict__ prow = jb.prow;
  double* __restrict__ inv = jb.inv;
  const int64_t w = 2 * (int64_t)n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = idx / n, m = idx - k * n;
    inv[k * n + prow[m]] = M[(int64_t)prow[k] * w + n + m];
  }
}

size_t dense_invert_work(int n) {
  // doubles: M (2n^2), F and Wc (n*GJB each), R (GJB*2*GJ_NB), Pinv (GJB^2), Yo and Rb (n*GJ_NB each);
  // then 16*GJB tournament candidates and 2n ints
  return (size_t)(2 * (int64_t)n * n + 2 * (int64_t)n * GJB + 2 * (int64_t)GJB * GJ_NB + GJB * GJB +
                  2 * (int64_t)n * GJ_NB) * sizeof(double) +
         (size_t)(16 * GJB + 2 * n) * sizeof(int);
}

GJJob gj_make_job(int n, const double* a, double* inv, double* work, int* status) {
  GJJob j;
  j.n = n;
  j.a = a;
  j.inv = inv;
  j.status = status;
  j.M = work;
  j.F = j.M + 2 * (int64_t)n * n;
  j.Wc = j.F + (int64_t)n * GJB;
  j.R = j.Wc + (int64_t)n * GJB;
  j.Pinv = j.R + 2 * (int64_t)GJB * GJ_NB;
  j.Yo = j.Pinv + GJB * GJB;
  j.Rb = j.Yo + (int64_t)n * GJ_NB;
  j.cand = (int*)(j.Rb + (int64_t)GJ_NB * n);
  j.done = j.cand + 16 * GJB;
  j.prow = j.done + n;
  return j;
}

// panel kernel variant of a size (0..3: RPT 1..4 rows per thread of 512 in
// registers, 4: tournament, 5: 5 rows per thread of 256)
constexpr int GJ_VARIANTS = 6;
int gj_variant(int n) {
  if (n > 4 * GJ_THREADS) return 4;
  if (n > 2 * GJ_THREADS && n <= 5 * 256) return 5;
  return (n - 1) / GJ_THREADS;
}

// The step loop over the widest job.  ns: job sizes in table order; groups:
// for each variant, its device selection list and size (single job: J.tab
// null, the job in `one`).
int gj_run(const GJJobs& J, const GJJob& one, const std::vector<int>& ns, const int* const groups[GJ_VARIANTS],
           const int gsize[GJ_VARIANTS], hipStream_t s) {
  const int nj = (int)ns.size();
  int nmax = 0;
  for (int n : ns) nmax = std::max(nmax, n);
  if (nmax > 16 * GJ_THREADS) return -1;  // at most 16 tournament blocks
  const dim3 zj(1024, 1, nj);
  gj_init_kernel<<<zj, 256, 0, s>>>(J, one);
  const int step = 16;  // every sub-panel width is a multiple
  for (int c0 = 0; c0 < nmax; c0 += GJ_NB) {
    for (int s0 = c0; s0 < std::min(nmax, c0 + GJ_NB); s0 += step) {
      bool any = false;
      for (int n : ns)
        any = any || (c0 < n && s0 < std::min(n, c0 + GJ_NB) && (s0 - c0) % gj_pbw(n) == 0);
      if (!any) continue;
      gj_fetch_kernel<<<dim3((nmax * GJB + 255) / 256, 1, nj), 256, 0, s>>>(J, one, c0, s0);
      for (int v = 0; v < GJ_VARIANTS; ++v) {
        if (!gsize[v]) continue;
        const GJJobs G{J.tab, groups[v]};
        switch (v) {
          case 0: gj_panel_kernel<1, 32, GJ_THREADS><<<dim3(1, 1, gsize[v]), GJ_THREADS, 0, s>>>(G, one, c0, s0); break;
          case 1: gj_panel_kernel<2, 32, GJ_THREADS><<<dim3(1, 1, gsize[v]), GJ_THREADS, 0, s>>>(G, one, c0, s0); break;
          case 2: gj_panel_kernel<3, 16, GJ_THREADS><<<dim3(1, 1, gsize[v]), GJ_THREADS, 0, s>>>(G, one, c0, s0); break;
          case 3: gj_panel_kernel<4, 16, GJ_THREADS><<<dim3(1, 1, gsize[v]), GJ_THREADS, 0, s>>>(G, one, c0, s0); break;
          case 5: gj_panel_kernel<5, 16, 256><<<dim3(1, 1, gsize[v]), 256, 0, s>>>(G, one, c0, s0); break;
          default:
            gj_tourn0_kernel<<<dim3(16, 1, gsize[v]), GJ_THREADS, 0, s>>>(G, one, c0, s0);
            gj_tourn1_kernel<<<dim3(1, 1, gsize[v]), GJ_THREADS, 0, s>>>(G, one, c0, s0);
        }
      }
      gj_rows_kernel<<<dim3((2 * GJ_NB + 255) / 256, GJB, nj), 256, 0, s>>>(J, one, c0, s0);
      gj_update_kernel<<<dim3((2 * GJ_NB + 255) / 256, (nmax + UPR - 1) / UPR, nj), 256, 0, s>>>(J, one, c0, s0);
    }
    gj_gather_kernel<<<dim3(1024, 1, nj), 256, 0, s>>>(J, one, c0);
    gj_gemm_kernel<<<dim3((nmax + GT - 1) / GT, (nmax + GT - 1) / GT, nj), 256, 0, s>>>(J, one, c0);
  }
  gj_extract_kernel<<<zj, 256, 0, s>>>(J, one);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// a: n x n input (not modified); inv: n x n output; work: dense_invert_work(n) bytes.
int dense_invert(int n, double* a, double* inv, double* work, int* status, hipStream_t s) {
  const GJJob one = gj_make_job(n, a, inv, work, status);
  const int* groups[GJ_VARIANTS] = {};
  int gsize[GJ_VARIANTS] = {};
  gsize[gj_variant(n)] = 1;
  return gj_run(GJJobs{nullptr, nullptr}, one, std::vector<int>{n}, groups, gsize, s);
}

// Batched: job tables built by dense_invert_batch_setup (device memory the
// caller owns); sizes in table order.
int dense_invert_batch(const GJJob* tab_dev, const int* sel_dev, const std::vector<int>& ns, hipStream_t s) {
  const int* groups[GJ_VARIANTS];
  int gsize[GJ_VARIANTS] = {};
  for (int n : ns) gsize[gj_variant(n)]++;
  int off = 0;
  for (int v = 0; v < GJ_VARIANTS; ++v) {
    groups[v] = sel_dev + off;
    off += gsize[v];
  }
  GJJob dummy{};
  return gj_run(GJJobs{tab_dev, nullptr}, dummy, ns, groups, gsize, s);
}

// host-side selection lists for dense_invert_batch: job indices grouped by variant
std::vector<int> dense_invert_batch_selection(const std::vector<int>& ns) {
  std::vector<int> sel;
  for (int v = 0; v < GJ_VARIANTS; ++v)
    for (int i = 0; i < (int)ns.size(); ++i)
      if (gj_variant(ns[i]) == v) sel.push_back(i);
  return sel;
}

// x = Ainv b on the coarsest level; one wavefront per output unknown, FP64
// accumulation; b and x are level vectors (component-major, padded).
template <typename T>
__device__ __forceinline__ void coarse_solve_body(const Grid& g, const double* __restrict__ Ainv,
                                                  const T* __restrict__ b, T* __restrict__ x, int bid) {
  const int64_t nd = (int64_t)NDOF * g.N;
  const int row = bid * 4 + (threadIdx.x >> 6);
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
__global__ void __launch_bounds__(256) coarse_solve_kernel(Grid g, const double* __restrict__ Ainv,
                                                           const T* __restrict__ b, T* __restrict__ x) {
  coarse_solve_body<T>(g, Ainv, b, x, blockIdx.x);
}
template <typename T>
__global__ void __launch_bounds__(256) coarse_solve_batch(const BJob* __restrict__ jobs, int njobs) {
  int bid;
  const BJob& j = find_job(jobs, njobs, bid);
  coarse_solve_body<T>(j.g, (const double*)j.A, (const T*)j.b, (T*)j.y, bid);
}

template <typename T>
void launch_coarse_solve(const Grid& g, const double* Ainv, const T* b, T* x, hipStream_t s) {
  const int64_t nd = (int64_t)NDOF * g.N;
  coarse_solve_kernel<T><<<(int)((nd + 3) / 4), 256, 0, s>>>(g, Ainv, b, x);
}
template void launch_coarse_solve<float>(const Grid&, const double*, const float*, float*, hipStream_t);
template void launch_coarse_solve<double>(const Grid&, const double*, const double*, double*, hipStream_t);

template <typename T>
void launch_coarse_solve_batch(const BJob* jobs, int njobs, int blocks, hipStream_t s) {
  coarse_solve_batch<T><<<blocks, 256, 0, s>>>(jobs, njobs);
}
template void launch_coarse_solve_batch<float>(const BJob*, int, int, hipStream_t);
template void launch_coarse_solve_batch<double>(const BJob*, int, int, hipStream_t);

}  // namespace mvpf
