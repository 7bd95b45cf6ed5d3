// Internal declarations of the mvpf library (not part of the C ABI).
//
// Data layout in HBM:
//  * vectors: structure-of-arrays, component-major: v[c * Npad + n] for the
//    NDOF = 3 + N unknowns c of node n (N variants: 9 for N = 6, 15 for
//    N = 12); Npad = N rounded up to 64; padding is kept 0.
//  * state:   3 + 2N FP64 components [u_x,u_y,u_z, eta_1..N, eta_n_1..N] in the
//    same SoA layout.
//  * NDOF x NDOF block operators on the structured 27-point stencil, symmetric half
//    storage, tiled: slice (t, u) = A + (t * 14 + u) * Lay<T>::SLICE holds the
//    block coupling node n = 64 t + l with its neighbour n + off(13 + u); entry
//    e = NDOF*row + col of lane l sits at Lay<T>::off(e, l), i.e. each lane's
//    entries come in groups of V = 16 / sizeof(T) (one 16-byte load), and the
//    64 lanes' groups are contiguous (one 1 KB coalesced wavefront load).
//    s = (dz+1)*9 + (dy+1)*3 + (dx+1) numbers the 27
//    offsets and s >= 13 are the diagonal and the 13 offsets with a positive
//    node-index difference.  The operator is symmetric (a Hessian, with
//    symmetric Dirichlet elimination), so the block for offset s < 13 is the
//    transpose of the stored block (n + off(s), 26 - s).  Blocks of
//    out-of-grid neighbours and of padding rows are zero.
//  * element matrices during assembly: E[(p * 81 + e) * NEpad + el] for the
//    36 node pairs p = (a <= b) of element el.
//  * diagonal blocks and their inverses: slice t = D + t * Lay<T>::SLICE, same
//    entry layout.
//  * per-Gauss-point scratch: qp[(comp * 8 + g) * NEpad + e].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mvpf.h"
#include "local.h"

namespace mvpf {

constexpr int NDOF = 3 + NV;         // unknowns per node: u (3), eta_hat (N)
constexpr int NSTATE = 3 + 2 * NV;   // state per node: u, eta_hat, eta_hat_n
constexpr int NSTEN = 27;
constexpr int NUP = 14;              // stored stencil blocks per row (diagonal + 13 upper)

// Lane exchange by a DPP control word (quad permutations, row mirrors): the
// value of the lane the control selects, moved through the VALU (no LDS).
// Every lane of these permutations has a source lane, so the bound control
// changes nothing; it lets the compiler fold the move into the VALU
// instruction that consumes it (a DPP source operand).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_t(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_t(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)u), hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// the value of lane `lane` in every lane (a scalar register read)
__device__ __forceinline__ double read_lane(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
constexpr int NPAIR = 36;            // element node pairs a <= b
constexpr int NBLK = NDOF * NDOF;
constexpr int TILE = 64;
constexpr int QP_GRAD = NQ;          // gradient components per Gauss point
constexpr int QP_HESS = NQ + NHP;    // gradient + packed Hessian
// packed Hessian entries rounded up to whole 8-component groups: the
// element-matrix kernel stages them 8 at a time, so the Gauss-point buffer
// holds NQ + NHP_PAD components (the padding is never used)
constexpr int NHP_PAD = (NHP + 7) / 8 * 8;
constexpr int QP_HESS_ALLOC = NQ + NHP_PAD;
constexpr int MAX_LEVELS = 8;
constexpr int MAX_RESTART = 64;
constexpr int SMALL_GRID_NODES = 10000;  // default size limit of the small-grid kernels
constexpr int BATCH_SMALL_GRID_NODES = 0;  // its default for the problems of a batch

struct Grid {
  int nx, ny, nz;      // elements
  int nnx, nny, nnz;   // nodes per direction
  int N;               // nodes
  int Npad;            // nodes rounded up to TILE
  int ntiles;
  int NE, NEpad;       // elements, rounded up to TILE
  double h;
};

Grid make_grid(int nx, int ny, int nz, double h);

// A slab of the assembly: elements e0 .. e0 + NEc - 1 (whole element layers,
// stored at local index e - e0 in the Gauss-point and element-matrix
// buffers, padded to NEcpad) feed node rows n0 .. n1 - 1 (whole node layers;
// the last slab also owns the padding rows up to Npad).  Slabs of one level
// overlap by one element layer, which is assembled twice.
struct Chunk {
  int64_t e0;
  int NEc, NEcpad;
  int n0, n1;
};
// Slabs of at most ne_cap padded elements each (one slab if the level fits).
std::vector<Chunk> make_chunks(const Grid& g, int64_t ne_cap);

// Logical block index with the 8 XCDs of the chip in mind: hardware places
// workgroup b on XCD b % 8; consecutive logical ids are kept on one XCD so
// that neighbouring tiles share its L2 (nb_pad: the grid, a multiple of 8).
__device__ __forceinline__ int xcd_logical(int b, int nb_pad) {
  const int per = nb_pad >> 3;
  return (b & 7) * per + (b >> 3);
}

// element node pair a <= b < 8 -> 0..35, and back
__host__ __device__ constexpr int pair_index(int a, int b) { return a * 8 - (a * (a - 1)) / 2 + (b - a); }
__host__ __device__ constexpr int pair_a(int p) { return p < 8 ? 0 : p < 15 ? 1 : p < 21 ? 2 : p < 26 ? 3 : p < 30 ? 4 : p < 33 ? 5 : p < 35 ? 6 : 7; }
__host__ __device__ constexpr int pair_b(int p) { return pair_a(p) + p - pair_index(pair_a(p), pair_a(p)); }

// Matrix-free finest level: Gauss-point Hessian entry k (packed upper
// triangle, 0..119) of point g of element e in storage type T.  Hessian
// entries come in groups of V = 16 / sizeof(T) per lane (one 16-byte load)
// and 64 lanes (8 elements x 8 points) per group, so a wavefront reads 1 KB
// contiguous (and, wave-contiguous, the 8 elements' 120 x 64 entries in one
// span).
template <typename T>
__host__ __device__ inline int64_t mf_index(int64_t NEpad, int k, int g, int64_t e) {
  constexpr int V = 16 / (int)sizeof(T);
  return ((((e >> 3) * (NHP / V) + k / V) * 64) + g * 8 + (e & 7)) * V + k % V;
}

// Element outputs of the matrix-free product, merged along x.  A node with
// offset (by, bz) in the element row r = ey + ny ez (node row j = ey + by,
// k = ez + bz) receives, from that row, the left-corner part of element
// (i, r) and the right-corner part of element (i - 1, r).  The element kernel
// adds the two when both elements belong to its workgroup (epw consecutive
// elements, epw = 8, 16 or 32) and stores per element e, q = by + 2 bz and
// unknown c:
//   L[(9q + c) NEpad + e]   left part of e (+ right part of e - 1 if merged)
//   W[(9q + c) NW + w]      right part of workgroup w's last element, unless
//                           it ends its row (the next workgroup's first
//                           element then reads it)
//   Rr[(9q + c) NR + r]     right part of row r's last element
// and the face outputs of penalty contact (3 values per face corner a =
// bx + 2 by, per top face f = fi + nx fj):
//   Cf[(3a + c) NF + f]
// Half the element-indexed values of a store per corner; the two parts of a
// node meet in one addition, in the kernel or in the gather, so the sums do
// not depend on epw.
__host__ __device__ inline int mf_epw_of(int epw) { return (epw == 8 || epw == 16) ? epw : 32; }
__host__ __device__ inline int64_t mf_nw(const Grid& g) { return (int64_t)g.NEpad / 8; }
__host__ __device__ inline int64_t mf_nr(const Grid& g) { return ((int64_t)g.ny * g.nz + 63) / 64 * 64; }
__host__ __device__ inline int64_t mf_nf(const Grid& g) { return ((int64_t)g.nx * g.ny + 63) / 64 * 64; }
__host__ __device__ inline int64_t mf_w_offset(const Grid& g) { return (int64_t)36 * g.NEpad; }
__host__ __device__ inline int64_t mf_r_offset(const Grid& g) { return mf_w_offset(g) + 36 * mf_nw(g); }
__host__ __device__ inline int64_t mf_cf_offset(const Grid& g) { return mf_r_offset(g) + 36 * mf_nr(g); }
__host__ __device__ inline int64_t mf_out_values(const Grid& g) { return mf_cf_offset(g) + 12 * mf_nf(g); }

// Rigid spherical indenter: centre (cx, cy, cz), radius R, contact penalty eps.
struct Sphere {
  double cx, cy, cz, R, eps;
};

// Entry layout inside a 64-lane block slice (see the file comment).
template <typename T>
struct Lay {
  static constexpr int V = 16 / (int)sizeof(T);                 // entries per 16-byte load
  static constexpr int NE = (NBLK + V - 1) / V * V;             // padded entries per lane
  static constexpr int NQ = NE / V;                             // 16-byte loads per block
  static constexpr int64_t SLICE = (int64_t)NE * TILE;
  __host__ __device__ static constexpr int64_t off(int e, int l) { return ((int64_t)(e / V) * TILE + l) * V + e % V; }
};

// Packed symmetric block (upper triangle, row-major, r <= c) in the same
// slice layout: the FP32 block inverses of a matrix-free finest level.
constexpr int NSYM = NDOF * (NDOF + 1) / 2;
__host__ __device__ constexpr int sym_index(int r, int c) {
  return r <= c ? r * NDOF - r * (r - 1) / 2 + (c - r) : c * NDOF - c * (c - 1) / 2 + (r - c);
}
template <typename T>
struct LaySym {
  static constexpr int V = 16 / (int)sizeof(T);
  static constexpr int NE = (NSYM + V - 1) / V * V;
  static constexpr int64_t SLICE = (int64_t)NE * TILE;
  __host__ __device__ static constexpr int64_t off(int e, int l) { return ((int64_t)(e / V) * TILE + l) * V + e % V; }
};

template <typename T>
struct Vec16;
template <>
struct Vec16<float> { typedef float4 type; };
template <>
struct Vec16<double> { typedef double2 type; };

struct Level {
  Grid g;
  double* state = nullptr;    // [NSTATE][Npad]
  uint16_t* mask = nullptr;   // [Npad] constrained-dof bits (bit c = dof c)
  double* target = nullptr;   // [Npad] prescribed u_z on the top face (finest only)
  double* A64 = nullptr;      // FP64 operator (finest; every level in FP64 mode)
  float* A32 = nullptr;       // FP32 operator (mixed mode, all but coarsest)
  double* diag64 = nullptr;   // FP64 diagonal blocks [ntiles][NBLK][64]
  double* Dinv64 = nullptr;   // FP64 block inverses (FP64 mode)
  float* Dinv32 = nullptr;    // FP32 block inverses (mixed mode)
  float* DinvS32 = nullptr;   // their upper triangles, packed (matrix-free finest level, mixed mode)
  // work vectors of the V-cycle (type per precision mode), [9][Npad]
  void* x = nullptr;
  void* x2 = nullptr;
  void* b = nullptr;
  void* r = nullptr;
  // coarsest level: dense inverse in SoA dof order (9 * N)^2
  double* Ainv = nullptr;
  int ndense = 0;
};

struct KernelTimer {
  std::vector<hipEvent_t> ev;  // start/stop pairs
  int used = 0;
  int launches = 0;
  double total_ms = 0.0;
  double bytes = 0.0;
};

}  // namespace mvpf

namespace mvpf {
// coarsest levels up to this many unknowns are inverted on a side stream,
// overlapping the assembly of the finer levels (all sizes: measured faster
// than in order at 1 125 and 6 561 unknowns)
constexpr int COARSE_OVERLAP_MAX = MVPF_MAX_COARSE_DOF;
// most blocks of a two-stage reduction (partials per reduced value)
constexpr int MAX_RED_BLOCKS = 4096;
// assembly buffers: the whole finest level up to this size, else slabs
constexpr int64_t ASSEMBLY_FULL_MAX = (int64_t)96 << 30;
constexpr int64_t ASSEMBLY_SLAB_BYTES = (int64_t)40 << 30;
}  // namespace mvpf

struct mvpf_problem {
  mvpf_mesh mesh;
  mvpf_material mat;                 // six-variant card (orbit == false)
  mvpf_orbit_material omat;          // card from one stretch tensor's cubic orbit (orbit == true)
  bool orbit = false;
  mvpf_loading load;
  mvpf_opts opts;
  int restart_cap = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int L = 0;
  bool mixed = false;
  mvpf::Level lev[mvpf::MAX_LEVELS];
  mvpf::DevCard* card = nullptr;     // device copy
  int pade = 22;                     // Pade order of the Hencky strain (11, 22, 33)
  int mixing = 0;                    // MVPF_MIX_LINEAR or MVPF_MIX_LOG
  double* qp = nullptr;              // per-Gauss-point scratch (finest size)
  double* elem = nullptr;            // element matrices, upper node pairs (finest size)
  void* Cbuf = nullptr;              // lower-half contributions, 13 * NDOF * Npad doubles (finest size)
  // matrix-free finest level (tuning key "matrix_free"): Gauss-point Hessians
  // in the matrix-free layout, FP64 (outer product, FP64 mode) and FP32
  // (mixed-mode smoother); element outputs go to Cbuf
  int mf = mvpf::NV == 6 ? 1 : 0;    // the matrix-free finest level exists for six variants
  int mf_epw = 32;                   // elements per workgroup of the matrix-free element kernel (8, 16, 32)
  double* Dmf64 = nullptr;
  float* Dmf32 = nullptr;
  mvpf::Sphere* sphere = nullptr;    // the indenter of the current system (device), sphere contact only
  double depth = 0.0;                // depth of the current state
  double sys_depth = 0.0;            // depth used by the last Newton system
  bool have_system = false;
  bool have_solution = false;
  // Newton / Krylov vectors (finest level, FP64 unless noted), [9][Npad]
  double* R = nullptr;       // residual
  double* rhs = nullptr;     // Newton right-hand side
  double* gvec = nullptr;    // prescribed increment (lifting)
  double* dx = nullptr;      // solution of the last solve
  double* tmp = nullptr;     // work
  double* tmp2 = nullptr;
  double* V = nullptr;       // (m+1) basis vectors
  void* Z = nullptr;         // m preconditioned vectors (FP32 in mixed mode)
  double* red = nullptr;     // reduction partials
  double* hcol = nullptr;    // device column of H (m+2)
  double* hhost = nullptr;   // pinned host mirror
  double* save_state = nullptr;  // backup for step rejection
  int64_t bytes = 0;
  bool timing = false;
  int row_G[mvpf::MAX_LEVELS] = {0};  // launch shape of the smoother/defect kernels per level
  int outer_G = 0;                     // launch shape of the outer FP64 operator product
  int small_nodes = mvpf::SMALL_GRID_NODES;  // levels up to this size use the small-grid kernels
  int tune_cache_use = 1;                    // mvpf_autotune reuses results for the same shapes
  mvpf::KernelTimer t_sweep, t_outer, t_resid, t_qp;
  // the coarsest-level inversion runs on a second stream (default priority),
  // overlapping the assembly of the finer levels
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* coarse_work = nullptr;     // dense scratch when V is too small
  bool coarse_pending = false;
  int coarse_overlap = -1;           // 1: side stream, 0: problem stream, -1: by size
  // Galerkin coarse levels (opts.coarse): element matrices of level l >= 1,
  // [(p * NBLK + q) * NEpad_l + E], allocated on first use
  double* gal[mvpf::MAX_LEVELS] = {nullptr};
  int64_t ne_cap = 0;                // element capacity of qp / elem (assembly slab size)
  int64_t ne_use = 0;                // slab size in use (<= ne_cap)
  int config_version = 0;            // bumped by set_opts / set_tuning / autotune (captured graphs)
};

namespace mvpf {

// ---- launchers (all asynchronous on `s`) ----------------------------------
// quadrature / assembly
void launch_qp(const Grid& g, const Chunk& ck, const double* state, const DevCard* cd, int pade, int mixing,
               double* qp, bool hess, hipStream_t s);
void launch_residual_gather(const Grid& g, const Chunk& ck, const double* state, const double* qp, const DevCard* cd,
                            double* R, hipStream_t s);
// diag_only: only the 8 diagonal node pairs / the diagonal blocks (the
// matrix-free finest level needs nothing else)
void launch_element_matrices(const Grid& g, const Chunk& ck, const double* qp, const DevCard* cd, double* elem,
                             hipStream_t s, bool diag_only = false);
void launch_jacobian_gather(const Grid& g, const Chunk& ck, const double* elem, double* A64, float* A32, double* diag64,
                            hipStream_t s, bool diag_only = false);
void launch_apply_dirichlet(const Grid& g, const uint16_t* mask, double* A64, float* A32, double* diag64,
                            hipStream_t s);
// Galerkin coarsening (galerkin.hip): element matrices of the parent layers
// Z0 .. Z1 - 1 of level gp from the child element matrices Ec of chunk ckc of
// level gc (which must hold both child layers of each) and the child level's
// constrained-dof masks; parents go to Ep (whole level, stride gp.NEpad)
void launch_galerkin_coarsen(const Grid& gc, const Chunk& ckc, const double* Ec, const uint16_t* maskc,
                             const Grid& gp, int Z0, int Z1, double* Ep, hipStream_t s);
// block inverses of the diagonal blocks (outputs may be null; DinvS32: packed
// upper triangles in FP32)
void launch_block_inverse(const Grid& g, const double* diag64, double* Dinv64, float* Dinv32, float* DinvS32,
                          int* status, hipStream_t s);
// penalty contact with a rigid sphere (MVPF_LOAD_SPHERE)
Sphere make_sphere(const Grid& g, const mvpf_loading& ld, double depth);
void launch_contact_residual(const Grid& g, const Sphere& sp, const double* state, double* R, hipStream_t s);
// adds the face stiffness to the element matrices if the chunk holds the top
// element layer (diagonal node pairs only when diag_only)
void launch_contact_element(const Grid& g, const Chunk& ck, const Sphere& sp, const double* state, double* elem,
                            hipStream_t s, bool diag_only = false);
void launch_contact_load(const Grid& g, const Sphere& sp, const double* state, double* out, hipStream_t s);
// matrix-free contact stiffness: the face outputs K_c x of every top face
// (zero without contact) into the contact part of the element-output buffer
// E; sp: the indenter in device memory
template <typename T, typename TX>
void launch_contact_apply(const Grid& g, const Sphere* sp, const double* state, const uint16_t* mask, const TX* x, T* E,
                          hipStream_t s);
// matrix-free finest level (mf.hip): laid out for the six-variant card
constexpr bool MF_AVAILABLE = NV == 6;
size_t mf_hessian_values(const Grid& g);
void launch_mf_pack(const Grid& g, const Chunk& ck, const double* qp, double* D64, float* D32, hipStream_t s);
template <typename TD, typename TX, typename T>
// elems_per_wg: elements per workgroup (8, 16 or 32 = 64, 128 or 256 threads)
void launch_mf_element(const Grid& g, const TD* D, const TX* x, const uint16_t* mask, const DevCard* cd, T* E,
                       hipStream_t s, bool sparse_x = false, int elems_per_wg = 32);
// MODE 0: y = K x; 1: y = b - K x; 2: y = x + omega Dinv (b - K x); constrained rows act as the identity.
// E: outputs of launch_mf_element with the same elems_per_wg (and of
// launch_contact_apply when contact)
template <int MODE, typename T, typename TX, typename TY>
void launch_mf_gather(const Grid& g, const T* E, bool contact, int elems_per_wg, const uint16_t* mask, const TX* x,
                      const T* b, const T* Dinv, T omega, TY* y, hipStream_t s);
// BSR products (TA = operator type, TX = vector type)
// G: number of workgroups (0 = one per 256 rows; smaller = persistent rounds).
// C: scratch for the transposed lower-half contributions, >= 13 * 9 * Npad
// values of the accumulation type (TY for spmv, T otherwise).
template <typename TA, typename TX, typename TY>
void launch_spmv(const Grid& g, const TA* A, const TX* x, TY* y, void* C, hipStream_t s, int G = 0);
template <typename T>
void launch_defect(const Grid& g, const T* A, const T* x, const T* b, T* r, void* C, hipStream_t s, int G = 0);
template <typename T>
void launch_pbj(const Grid& g, const T* A, const T* Dinv, const T* x, const T* b, T* xo, T omega,
                bool zero_guess, void* C, hipStream_t s, int G = 0);
// coarse-level variant (27 threads per row); out = b - A x, or the damped
// point-block Jacobi update when pbj is set.  Used on levels with at most
// small_grid_nodes nodes (default SMALL_GRID_NODES, a tuning key).
template <typename T>
void launch_row_small(const Grid& g, const T* A, const T* Dinv, const T* x, const T* b, T* out, T omega, bool pbj,
                      hipStream_t s);
// transfers
template <typename T>
void launch_restrict(const Grid& fine, const Grid& coarse, const T* rf, const uint16_t* cmask, T* bc,
                     hipStream_t s);
template <typename T>
void launch_prolong_add(const Grid& fine, const Grid& coarse, const T* ec, const uint16_t* fmask, T* xf,
                        hipStream_t s);
void launch_inject(const Grid& fine, const Grid& coarse, const double* sf, double* sc, hipStream_t s);
void launch_inject_mask(const Grid& fine, const Grid& coarse, const uint16_t* mf, uint16_t* mc,
                        hipStream_t s);
// coarse direct solve
void launch_dense_from_bsr(const Grid& g, const double* A64, double* dense, hipStream_t s);
size_t dense_invert_work(int n);  // bytes of scratch needed by dense_invert
// one dense inversion: pointers into its dense_invert_work(n) workspace
struct GJJob {
  int n;
  const double* a;  // input n x n (not modified)
  double* inv;      // output n x n
  double *M, *F, *Wc, *R, *Pinv, *Yo, *Rb;
  int *cand, *done, *prow;
  int* status;
};
GJJob gj_make_job(int n, const double* a, double* inv, double* work, int* status);
// several inversions at once: tab_dev = device table of jobs, sel_dev =
// device copy of dense_invert_batch_selection(ns), ns = job sizes
int dense_invert_batch(const GJJob* tab_dev, const int* sel_dev, const std::vector<int>& ns, hipStream_t s);
std::vector<int> dense_invert_batch_selection(const std::vector<int>& ns);
int dense_invert(int n, double* a, double* inv, double* work, int* piv_status, hipStream_t s);
template <typename T>
void launch_coarse_solve(const Grid& g, const double* Ainv, const T* b, T* x, hipStream_t s);
// vectors
void launch_interleaved_to_soa(const Grid& g, const double* in, int ncomp, int comp0, int ldc,
                               double* out, hipStream_t s);
void launch_soa_to_interleaved(const Grid& g, const double* in, int ncomp, int comp0, int ldc,
                               double* out, hipStream_t s);
template <typename TI, typename TO>
void launch_convert_masked(const Grid& g, const TI* in, const uint16_t* mask, TO* out, hipStream_t s);
void launch_set_constrained(const Grid& g, const uint16_t* mask, const double* src, double* dst,
                            hipStream_t s);
void launch_dirichlet_masks(const Grid& g, const mvpf_loading& ld, double depth, uint16_t* mask,
                            double* target, hipStream_t s);
void launch_increment(const Grid& g, const uint16_t* mask, const double* target, const double* state,
                      double* gvec, hipStream_t s);
void launch_newton_rhs(const Grid& g, const uint16_t* mask, const double* R, const double* Kg,
                       const double* gvec, double* rhs, hipStream_t s);
void launch_state_update(const Grid& g, const uint16_t* mask, const double* target, const double* dx,
                         double* state, hipStream_t s);
void launch_init_random(const Grid& g, uint64_t seed, double* state, hipStream_t s);
void launch_free_norm_partial(const Grid& g, const double* v, const uint16_t* mask, double* part,
                              hipStream_t s);
// Krylov (n = 9 * Npad)
int red_blocks(int64_t n);
void launch_multidot(int64_t n, const double* V, int64_t ldv, int k, const double* w, double* part,
                     hipStream_t s);
void launch_reduce(int k, int nblk, const double* part, double* out, int accumulate, hipStream_t s);
void launch_multiaxpy(int64_t n, const double* V, int64_t ldv, int k, const double* h, double* w,
                      double* part_norm, hipStream_t s);
// w -= sum_j h_j V_j, then part = the block partial sums of V_j . w (the
// updated w), j < k: multiaxpy followed by multidot, bitwise, in one sweep
// over the basis when k <= 32
void launch_multiaxpy_dot(int64_t n, const double* V, int64_t ldv, int k, const double* h, double* w, double* part,
                          hipStream_t s);
void launch_scale(int64_t n, const double* w, const double* beta, double* v, hipStream_t s);
template <typename TZ>
void launch_combine(int64_t n, const TZ* Z, int64_t ldz, int k, const double* y, double* x, hipStream_t s);
void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                  hipStream_t s);
template <typename T>
void launch_zero(int64_t n, T* p, hipStream_t s);
template <typename TI, typename TO>
void launch_convert(int64_t n, const TI* in, TO* out, hipStream_t s);
template <typename T, typename TZ>
void launch_precond_finish(const Grid& g, const T* x, const double* v, const uint16_t* mask, TZ* z, hipStream_t s);

// ---- batched launches: one launch of an operator for many problems -----------
// A job is one problem's part of a launch: its workgroups block0 ..
// block0 + nblk - 1.  The job table sits in device memory, sorted by block0;
// every workgroup finds its job by binary search.
struct BJob {
  Grid g;                  // the level (finest grid of a transfer)
  Grid g2;                 // coarse grid of a transfer
  const void* A;           // half-stencil operator, Gauss-point Hessians or dense coarse inverse
  const void* D;           // block inverses
  const void* x;           // input vector
  const void* b;           // right-hand side; FP64 vector v at the preconditioner's ends
  void* y;                 // output vector
  void* C;                 // scratch: transposed contributions or element outputs
  const uint16_t* mask;    // constrained-dof masks of the output's level
  const DevCard* cd;       // material card (matrix-free element kernel)
  double omega;            // damping of the Jacobi sweeps
  int block0, nblk;
  int epw;                 // matrix-free gathers: elements per workgroup of the element launch
  int contact;             // matrix-free gathers: add the contact face outputs
};
// job of this workgroup in a batched launch; bid = its workgroup index within the job
template <typename J>
__device__ inline const J& find_job(const J* __restrict__ jobs, int njobs, int& bid) {
  int lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (jobs[mid].block0 <= (int)blockIdx.x) lo = mid; else hi = mid;
  }
  bid = (int)blockIdx.x - jobs[lo].block0;
  return jobs[lo];
}
enum BatchOp {
  BOP_CONVERT,          // b = mask(v), FP64 -> T
  BOP_PBJ_ZERO,         // y = omega D^-1 b
  BOP_DEFECT_SPLIT,     // pass 1 of b - A x (y = partial, C = transposed contributions)
  BOP_PBJ_LOWER,        // pass 2, then y = x + omega D^-1 (b - A x)
  BOP_DEFECT_LOWER,     // pass 2 of y = b - A x
  BOP_ROW_SMALL_PBJ,    // small-grid Jacobi sweep
  BOP_ROW_SMALL_DEFECT, // small-grid defect
  BOP_RESTRICT,         // y (coarse) = masked P^T x (fine)
  BOP_PROLONG,          // y (fine) += P x (coarse), constrained dofs untouched
  BOP_COARSE,           // y = Ainv b (dense FP64 inverse)
  BOP_MF_ELEMENT,       // C = element parts of K x (matrix-free finest level)
  BOP_MF_GATHER_PBJ,    // y = x + omega D^-1 (b - sum C)
  BOP_MF_GATHER_DEFECT, // y = b - sum C
  BOP_FINISH,           // z = x, v on constrained dofs, T -> TZ
  BOP_MF_OUTER_ELEMENT, // C = element parts of K z (FP64 Hessians, z of type TZ)
  BOP_MF_OUTER_GATHER,  // y = sum C (FP64), constrained rows = z
};
// Batched Krylov vector operations (FGMRES of many problems in lockstep); a
// job's arithmetic is that of the single-problem launch (same partial-sum
// blocks), so results are bitwise the same.
struct KJob {
  int64_t n;           // vector length
  const double* V;     // basis vectors, leading dimension n
  double* w;           // the vector worked on
  double* part;        // partial sums
  const double* h;     // coefficients (multiaxpy)
  double* out;         // results (reduce), destination (copy)
  const double* src;   // source (copy)
  double a;            // factor (scale)
  int k;               // vectors (multidot, multiaxpy) or values (reduce, copy)
  int nb;              // partial sums per value (reduce)
  int flag;            // multiaxpy: norm partials into part; reduce: accumulate
  int block0, nblk;
};
enum KrylovOp {
  KOP_MULTIDOT,   // part[j][blk] = V_j . w over the block's chunk, j < k
  KOP_REDUCE,     // out[j] (+)= sum_b part[j][b], j < k
  KOP_MULTIAXPY,  // w -= sum_j h_j V_j (norm partials of w into part)
  KOP_SCALE,      // w = a w
  KOP_COPY,       // out[0..k) = src[0..k)
};
int krylov_job_blocks(int op, const KJob& j);
// Batched assembly of the Newton systems of many problems: one launch per
// assembly kernel and level for all problems (each a single slab).
struct AJob {
  Grid g;
  Chunk ck;
  const double* state;
  const DevCard* cd;
  double* qp;                // Gauss-point scratch
  double* elem;              // element matrices
  double *A64, *diag64, *Dinv64, *R, *D64;
  float *A32, *Dinv32, *D32, *DinvS32;
  const uint16_t* mask;
  int* status;
  int64_t eb0, neb;          // element groups of the Hessian pack
  int npair, nblocks, nup;   // pairs of the element matrices; gather blocks
  int block0, nblk;
};
constexpr int QP_LOG_MIX = 1000;  // added to the Pade order of a batched Hessian launch: logarithmic mixing
enum AssemblyOp {
  AOP_QP_HESS,        // Gauss-point gradients and Hessians (Pade order, + QP_LOG_MIX for log mixing)
  AOP_ELEMENT,        // element matrices (npair pairs)
  AOP_GATHER,         // stored blocks (nup per tile; A64 / A32 null: diagonal only)
  AOP_DIRICHLET,      // symmetric elimination on the stored blocks
  AOP_BLOCK_INVERSE,  // 9x9 diagonal-block inverses
  AOP_RESIDUAL,       // residual rows from the Gauss-point gradients
  AOP_MF_PACK,        // Gauss-point Hessians into the matrix-free layout
};
// fills the job's derived fields (npair, nblocks, nup, eb0, neb) and returns its workgroups
int assembly_job_blocks(int op, AJob& j, bool diag_only);
void launch_assembly_batch(int op, int pade, const AJob* jobs, int njobs, int blocks, hipStream_t s);
void launch_mf_pack_batch(const AJob* jobs, int njobs, int blocks, hipStream_t s);
int mf_pack_job_blocks(AJob& j);
void launch_krylov_batch(int op, const KJob* jobs, int njobs, int blocks, hipStream_t s);
template <typename TZ>
void launch_mf_outer_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s, int threads = 256);
// workgroups one job of op needs (threads: workgroup size of the
// matrix-free element kernels, 64, 128 or 256)
int batch_job_blocks(int op, const BJob& j, int threads = 256);
int bsr_job_blocks(int op, const Grid& g);
int mf_job_blocks(int op, const Grid& g, int threads = 256);
int vec_job_blocks(const Grid& g);
// T: multigrid precision; TZ: type of the preconditioned vector (BOP_FINISH)
template <typename T, typename TZ>
void launch_batch(int op, const BJob* jobs_dev, int njobs, int total_blocks, hipStream_t s, int threads = 256);
template <typename T>
void launch_bsr_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s);
template <typename T>
void launch_transfer_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s);
template <typename T>
void launch_coarse_solve_batch(const BJob* jobs, int njobs, int blocks, hipStream_t s);
template <typename T>
void launch_mf_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s, int threads = 256);
template <typename T, typename TZ>
void launch_vec_batch(int op, const BJob* jobs, int njobs, int blocks, hipStream_t s);

}  // namespace mvpf
