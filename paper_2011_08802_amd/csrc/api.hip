// C-ABI implementation: problem setup, Newton system assembly on all levels,
// the multigrid V-cycle, FGMRES and the Newton / time-step drivers.  Host code
// only orchestrates; every arithmetic step on the solve path runs in the HIP
// kernels of this library.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <string>

#include "common.h"

using namespace mvpf;

static thread_local std::string g_create_err;

namespace mvpf {

Grid make_grid(int nx, int ny, int nz, double h) {
  Grid g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.nnx = nx + 1; g.nny = ny + 1; g.nnz = nz + 1;
  g.N = g.nnx * g.nny * g.nnz;
  g.Npad = (g.N + TILE - 1) / TILE * TILE;
  g.ntiles = g.Npad / TILE;
  g.NE = nx * ny * nz;
  g.NEpad = (g.NE + TILE - 1) / TILE * TILE;
  g.h = h;
  return g;
}

std::vector<Chunk> make_chunks(const Grid& g, int64_t ne_cap) {
  std::vector<Chunk> out;
  if ((int64_t)g.NEpad <= ne_cap) {
    out.push_back(Chunk{0, g.NE, g.NEpad, 0, g.Npad});
    return out;
  }
  const int64_t nxy = (int64_t)g.nx * g.ny, nnxy = (int64_t)g.nnx * g.nny;
  const int L = (int)std::max<int64_t>((ne_cap - (TILE - 1)) / nxy - 1, 1);  // node layers per slab
  for (int k0 = 0; k0 < g.nnz; k0 += L) {
    const int k1 = std::min(k0 + L, g.nnz);
    const int ez0 = std::max(k0 - 1, 0), ez1 = std::min(k1, g.nz);
    Chunk c;
    c.e0 = ez0 * nxy;
    c.NEc = (int)((ez1 - ez0) * nxy);
    c.NEcpad = (c.NEc + TILE - 1) / TILE * TILE;
    c.n0 = (int)(k0 * nnxy);
    c.n1 = (k1 == g.nnz) ? g.Npad : (int)(k1 * nnxy);
    out.push_back(c);
  }
  return out;
}

}  // namespace mvpf

namespace {

#define HIPCHK(call)                                                             \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      p->err = std::string(#call) + " failed: " + hipGetErrorString(e_);         \
      return MVPF_EDEVICE;                                                       \
    }                                                                            \
  } while (0)

#define TRY(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ < 0) return rc_;   \
  } while (0)

int launch_check(mvpf_problem* p, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    p->err = std::string(where) + ": " + hipGetErrorString(e);
    return MVPF_EDEVICE;
  }
  return 0;
}

template <typename T>
int dalloc(mvpf_problem* p, T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return 0;
  const size_t bytes = count * sizeof(T);
  hipError_t e = hipMalloc((void**)ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    p->err = "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e);
    return MVPF_ENOMEM;
  }
  p->bytes += (int64_t)bytes;
  e = hipMemsetAsync(*ptr, 0, bytes, p->stream);
  if (e != hipSuccess) {
    p->err = std::string("hipMemsetAsync failed: ") + hipGetErrorString(e);
    return MVPF_EDEVICE;
  }
  return 0;
}

template <typename T>
void dfree(T*& ptr) {
  if (ptr) (void)hipFree((void*)ptr);
  ptr = nullptr;
}

// ---- material card (Sec. 4.1, Table 1), rotated into the sample frame ----
using T4 = double[3][3][3][3];

void voigt_to_t4(const double C[6][6], T4 L) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) L[i][j][k][l] = C[SI(i, j)][SI(k, l)];
}

void t4_to_voigt(const T4 L, double C[6][6]) {
  const int ia[6] = {0, 1, 2, 1, 0, 0}, ib[6] = {0, 1, 2, 2, 2, 1};
  for (int v = 0; v < 6; ++v)
    for (int u = 0; u < 6; ++u) C[v][u] = L[ia[v]][ib[v]][ia[u]][ib[u]];
}

// L'_ijkl = R_ia R_jb R_kc R_ld L_abcd
void rotate_t4(const T4 L, const double R[3][3], T4 out) {
  double t1[3][3][3][3], t2[3][3][3][3];
  for (int i = 0; i < 3; ++i)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          double s = 0;
          for (int a = 0; a < 3; ++a) s += R[i][a] * L[a][b][c][d];
          t1[i][b][c][d] = s;
        }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          double s = 0;
          for (int b = 0; b < 3; ++b) s += R[j][b] * t1[i][b][c][d];
          t2[i][j][c][d] = s;
        }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) {
          double s = 0;
          for (int c = 0; c < 3; ++c) s += R[k][c] * t2[i][j][c][d];
          t1[i][j][k][d] = s;
        }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double s = 0;
          for (int d = 0; d < 3; ++d) s += R[l][d] * t1[i][j][k][d];
          out[i][j][k][l] = s;
        }
}

// eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations:
// A = V diag(w) V^T (columns of V = eigenvectors)
void sym_eig3(const double A0[3][3], double w[3], double V[3][3]) {
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A[i][j] = A0[i][j];
      V[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    const double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
    const double scale = std::fabs(A[0][0]) + std::fabs(A[1][1]) + std::fabs(A[2][2]);
    if (off <= 1e-17 * scale) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        // rotation zeroing A[p][q] (Golub & Van Loan, symmetric Schur 2x2)
        const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- A J
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- J^T A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {  // V <- V J
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

// Card inputs in the cubic crystal frame, before the rotation Q into the
// sample frame: the austenite stiffness and each variant's stretch tensor
// and stiffness.
struct CubicCard {
  int n = 0;
  double U[NV][3][3];
  double L[NV][3][3][3][3];
  double L0[3][3][3][3];
};

// The rest of the card (Sec. 2.2-2.3, 3.1; Eqs. LinMix and IntEnergy, the
// logarithmic mixing rule of Sec. 2.1): everything rotated by Q, stored as
// differences to the austenite (U_k - I, L_k - L_0), log U_k for log
// mixing, chemical energies, the double-obstacle matrix and its condensed
// forms.
void fill_card(const CubicCard& cc, const double Qm[9], const double F0[NV + 1], double w_am, double w_mm, double ell,
               double rho, double eps, int pade, int mixing, DevCard& cd) {
  std::memset(&cd, 0, sizeof(cd));
  double Q[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Q[i][j] = Qm[3 * i + j];
  T4 L0s;
  rotate_t4(cc.L0, Q, L0s);
  double L0v[6][6];
  t4_to_voigt(L0s, L0v);
  for (int v = 0; v < NV; ++v) {
    double Us[3][3];  // Q U Q^T
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) s += Q[i][k] * cc.U[v][k][l] * Q[j][l];
        Us[i][j] = s;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) cd.dU[v][SI(i, j)] = Us[i][j] - (i == j ? 1.0 : 0.0);
    // log U_k = V diag(log w) V^T of the symmetric positive definite U_k
    double w[3], V[3][3];
    sym_eig3(Us, w, V);
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += V[i][k] * std::log(w[k]) * V[j][k];
        cd.logU[v][SI(i, j)] = s;
      }
    T4 Ls;
    rotate_t4(cc.L[v], Q, Ls);
    double Lv[6][6];
    t4_to_voigt(Ls, Lv);
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) cd.dL[v][i][j] = Lv[i][j] - L0v[i][j];
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) cd.L0[i][j] = L0v[i][j];
  for (int k = 0; k < NV; ++k) cd.dF0[k] = F0[k + 1] - F0[0];
  for (int i = 0; i <= NV; ++i)
    for (int j = 0; j <= NV; ++j) cd.W[i][j] = (i == j) ? 0.0 : ((i == 0 || j == 0) ? w_am : w_mm);
  // condensation eta_0 = 1 - sum eta_k: Hessian of 1/2 eta^T W eta w.r.t. eta_hat
  for (int k = 0; k < NV; ++k)
    for (int l = 0; l < NV; ++l) cd.Sw[k][l] = cd.W[k + 1][l + 1] - cd.W[k + 1][0] - cd.W[0][l + 1] + cd.W[0][0];
  // gradient energy -sum_{i<j} w_ij l^2 grad eta_i . grad eta_j in eta_hat
  const double l2 = ell * ell;
  for (int k = 0; k < NV; ++k)
    for (int l = 0; l < NV; ++l) {
      cd.Mg[k][l] = -l2 * cd.Sw[k][l];
      cd.Mg32[k][l] = (float)cd.Mg[k][l];
    }
  cd.rho = rho;
  cd.eps = eps;
  cd.pade = pade;
  cd.mixing = mixing;
}

// CuAlNi card (Sec. 4.1, Table 1; six variants): stretch tensors from
// alpha, beta, gamma; each variant's orthorhombic stiffness in the
// principal axes of its stretch tensor.  Valid for a library of six variants.
void build_card(const mvpf_material& m, DevCard& cd) {
  CubicCard cc;
  // austenite
  double C0[6][6] = {};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C0[a][b] = (a == b) ? m.cubic[0] : m.cubic[1];
  C0[3][3] = C0[4][4] = C0[5][5] = m.cubic[2];
  voigt_to_t4(C0, cc.L0);
  // martensite in its orthorhombic axes: c11,c22,c33,c44,c55,c66,c12,c13,c23
  const double* o = m.ortho;
  double Cm[6][6] = {};
  Cm[0][0] = o[0]; Cm[1][1] = o[1]; Cm[2][2] = o[2];
  Cm[3][3] = o[3]; Cm[4][4] = o[4]; Cm[5][5] = o[5];
  Cm[0][1] = Cm[1][0] = o[6];
  Cm[0][2] = Cm[2][0] = o[7];
  Cm[1][2] = Cm[2][1] = o[8];
  T4 Lmo;
  voigt_to_t4(Cm, Lmo);
  // variant k = 2*pair + sign: stretch tensor p(e_a e_a + e_b e_b) +- q (e_a e_b + e_b e_a)
  // + beta e_c e_c with p = (alpha+gamma)/2, q = (alpha-gamma)/2 (Sec. 4.1);
  // its alpha-, beta-, gamma-axes are (e_a +- e_b)/sqrt2, e_c, (e_a -+ e_b)/sqrt2.
  const int pa[3] = {0, 0, 1}, pb[3] = {2, 1, 2}, pc[3] = {1, 2, 0};
  const double pp = 0.5 * (m.alpha + m.gamma), qq = 0.5 * (m.alpha - m.gamma);
  const double r2 = 1.0 / std::sqrt(2.0);
  cc.n = NV < 6 ? NV : 6;
  for (int v = 0; v < cc.n; ++v) {
    const int pr = v / 2;
    const double sg = (v % 2 == 0) ? 1.0 : -1.0;
    const int a = pa[pr], b = pb[pr], c = pc[pr];
    double (&U)[3][3] = cc.U[v];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) U[i][j] = 0.0;
    U[a][a] = U[b][b] = pp;
    U[a][b] = U[b][a] = sg * qq;
    U[c][c] = m.beta;
    double R[3][3] = {};  // columns: alpha-, beta-, gamma-axis in crystal coordinates
    R[a][0] = r2; R[b][0] = sg * r2;
    R[c][1] = 1.0;
    R[a][2] = r2; R[b][2] = -sg * r2;
    rotate_t4(Lmo, R, cc.L[v]);
  }
  double F0[NV + 1] = {};
  for (int k = 0; k <= cc.n; ++k) F0[k] = m.F0[k];
  fill_card(cc, m.Q, F0, m.w_am, m.w_mm, m.ell, m.rho, m.eps_eta, m.pade, m.mixing, cd);
}

// The 24 rotations of the cube: signed permutation matrices of determinant
// +1, Q[i][perm[i]] = sign[i]; permutations in lexicographic order, then
// sign patterns with row 0's sign varying slowest, + before -.
int cubic_rotations(double out[24][3][3]) {
  int perm[3] = {0, 1, 2}, n = 0;
  do {
    for (int sgn = 0; sgn < 8; ++sgn) {
      double Q[3][3] = {};
      for (int i = 0; i < 3; ++i) Q[i][perm[i]] = ((sgn >> (2 - i)) & 1) ? -1.0 : 1.0;
      const double det = Q[0][0] * (Q[1][1] * Q[2][2] - Q[1][2] * Q[2][1]) -
                         Q[0][1] * (Q[1][0] * Q[2][2] - Q[1][2] * Q[2][0]) +
                         Q[0][2] * (Q[1][0] * Q[2][1] - Q[1][1] * Q[2][0]);
      if (det > 0) std::memcpy(out[n++], Q, sizeof(Q));
    }
  } while (std::next_permutation(perm, perm + 3));
  return n;
}

// Card of a material whose variants are the distinct images Q U1 Q^T of one
// stretch tensor under the cube's rotations (in the order above; images
// equal within 1e-12 are one variant), each with L1 rotated by the rotation
// that produced it.  Returns the number of variants the orbit has (the card
// is filled only if it equals the library's N).
int build_card_orbit(const mvpf_orbit_material& m, DevCard& cd) {
  CubicCard cc;
  double R[24][3][3];
  const int nr = cubic_rotations(R);
  double U1[3][3], L1v[6][6];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) U1[i][j] = m.U1[3 * i + j];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) L1v[i][j] = m.L1[6 * i + j];
  T4 L1;
  voigt_to_t4(L1v, L1);
  int n = 0;
  for (int r = 0; r < nr; ++r) {
    double V[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) s += R[r][i][k] * U1[k][l] * R[r][j][l];
        V[i][j] = s;
      }
    bool seen = false;
    for (int q = 0; q < (n < NV ? n : NV) && !seen; ++q) {
      double d = 0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) d = std::max(d, std::fabs(V[i][j] - cc.U[q][i][j]));
      seen = d <= 1e-12;
    }
    if (seen) continue;
    if (n < NV) {
      std::memcpy(cc.U[n], V, sizeof(V));
      rotate_t4(L1, R[r], cc.L[n]);
    }
    ++n;
  }
  if (n != NV) return n;
  cc.n = n;
  double C0[6][6] = {};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C0[a][b] = (a == b) ? m.cubic[0] : m.cubic[1];
  C0[3][3] = C0[4][4] = C0[5][5] = m.cubic[2];
  voigt_to_t4(C0, cc.L0);
  double F0[NV + 1];
  F0[0] = m.F0_a;
  for (int k = 1; k <= NV; ++k) F0[k] = m.F0_m;
  fill_card(cc, m.Q, F0, m.w_am, m.w_mm, m.ell, m.rho, m.eps_eta, m.pade, m.mixing, cd);
  return n;
}

// the problem's card (either kind), with the current viscous coefficient
void make_card(const mvpf_problem* p, DevCard& cd) {
  if (p->orbit)
    build_card_orbit(p->omat, cd);
  else
    build_card(p->mat, cd);
}

// ---- typed accessors for the two precision modes --------------------------
template <typename T> const T* opA(const Level& L);
template <> const float* opA<float>(const Level& L) { return L.A32; }
template <> const double* opA<double>(const Level& L) { return L.A64; }
template <typename T> const T* opD(const Level& L);
template <> const float* opD<float>(const Level& L) { return L.Dinv32; }
// block inverses read by the matrix-free finest level's Jacobi gather
template <typename T> const T* mfDinv(const Level& L);
template <> const double* mfDinv<double>(const Level& L) { return L.Dinv64; }
template <> const float* mfDinv<float>(const Level& L) { return L.DinvS32; }
template <> const double* opD<double>(const Level& L) { return L.Dinv64; }

int64_t nvec(const Grid& g) { return (int64_t)NDOF * g.Npad; }

void timer_begin(mvpf_problem* p, KernelTimer& t) {
  if (!p->timing) return;
  if ((int)t.ev.size() < 2 * (t.used + 1)) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    t.ev.push_back(a);
    t.ev.push_back(b);
  }
  (void)hipEventRecord(t.ev[2 * t.used], p->stream);
}

void timer_end(mvpf_problem* p, KernelTimer& t, double bytes) {
  if (!p->timing) return;
  (void)hipEventRecord(t.ev[2 * t.used + 1], p->stream);
  t.used++;
  t.bytes = bytes;
}

void timer_collect(mvpf_problem* p, KernelTimer& t) {
  if (t.used == 0) return;
  (void)hipStreamSynchronize(p->stream);
  for (int i = 0; i < t.used; ++i) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]);
    t.total_ms += ms;
    t.launches++;
  }
  t.used = 0;
}

// Exact count of in-grid (node, neighbour) pairs of the 27-point stencil, and
// of the stored half (diagonal + upper blocks) that the symmetric operator
// must read from memory.
double stencil_blocks(const Grid& g) {
  return (3.0 * g.nx + 1.0) * (3.0 * g.ny + 1.0) * (3.0 * g.nz + 1.0);
}
double stored_blocks(const Grid& g) { return 0.5 * (stencil_blocks(g) + g.N); }

// Algorithmic bytes of one damped point-block Jacobi sweep on level g:
// the operator (stored half-stencil blocks, or on a matrix-free level the
// 8 x 120 Gauss-point Hessian values per element), the block inverses, x, b
// and the new x.
template <typename T>
double sweep_bytes(const Grid& g, bool mf) {
  const double op = mf ? 960.0 * g.NE : stored_blocks(g) * NBLK;
  const double dinv = (mf && sizeof(T) == 4) ? NSYM : NBLK;  // packed symmetric FP32 inverses
  return sizeof(T) * (op + (double)g.N * (dinv + 3 * NDOF));
}

// ---- matrix-free finest level --------------------------------------------------
bool use_mf(const mvpf_problem* p) { return p->mf && p->Dmf64; }
bool contact(const mvpf_problem* p);
template <typename T> const T* mfD(const mvpf_problem* p);
template <> const float* mfD<float>(const mvpf_problem* p) { return p->Dmf32; }
template <> const double* mfD<double>(const mvpf_problem* p) { return p->Dmf64; }

// element outputs of K x on the finest level (x masked on constrained dofs
// when masked), contact stiffness included (indenter of the last
// build_system), into Cbuf; sparse: x is zero on most elements
template <typename T, typename TX>
void mf_elements(mvpf_problem* p, const TX* x, bool masked, bool sparse = false) {
  Level& L0 = p->lev[0];
  const uint16_t* mask = masked ? L0.mask : nullptr;
  launch_mf_element<T, TX, T>(L0.g, mfD<T>(p), x, mask, p->card, (T*)p->Cbuf, p->stream, sparse, p->mf_epw);
  if (contact(p)) launch_contact_apply<T, TX>(L0.g, p->sphere, L0.state, mask, x, (T*)p->Cbuf, p->stream);
}

// ---- V-cycle ------------------------------------------------------------------
template <typename T>
void sweep(mvpf_problem* p, int l, bool zero) {
  Level& L = p->lev[l];
  const T om = (T)p->opts.omega;
  const bool timed = (l == 0 && !zero);
  if (timed) timer_begin(p, p->t_sweep);
  if (!zero && l == 0 && use_mf(p)) {
    mf_elements<T, T>(p, (const T*)L.x, true);
    launch_mf_gather<2, T, T, T>(L.g, (const T*)p->Cbuf, contact(p), p->mf_epw, L.mask, (const T*)L.x, (const T*)L.b,
                                 mfDinv<T>(L), om, (T*)L.x2, p->stream);
  } else if (!zero && L.g.N <= p->small_nodes)
    launch_row_small<T>(L.g, opA<T>(L), opD<T>(L), (const T*)L.x, (const T*)L.b, (T*)L.x2, om, true, p->stream);
  else
    launch_pbj<T>(L.g, opA<T>(L), opD<T>(L), (const T*)L.x, (const T*)L.b, (T*)L.x2, om, zero, p->Cbuf, p->stream,
                  p->row_G[l]);
  if (timed) timer_end(p, p->t_sweep, sweep_bytes<T>(L.g, use_mf(p)));
  std::swap(L.x, L.x2);
}

template <typename T>
void vcycle(mvpf_problem* p, int l) {
  Level& L = p->lev[l];
  hipStream_t s = p->stream;
  if (l == p->L - 1) {
    launch_coarse_solve<T>(L.g, L.Ainv, (const T*)L.b, (T*)L.x, s);
    return;
  }
  if (p->opts.nu_pre > 0) {
    sweep<T>(p, l, true);
    for (int k = 1; k < p->opts.nu_pre; ++k) sweep<T>(p, l, false);
  } else {
    launch_zero<T>(nvec(L.g), (T*)L.x, s);
  }
  if (l == 0 && p->timing) timer_begin(p, p->t_resid);
  if (l == 0 && use_mf(p)) {
    mf_elements<T, T>(p, (const T*)L.x, true);
    launch_mf_gather<1, T, T, T>(L.g, (const T*)p->Cbuf, contact(p), p->mf_epw, L.mask, (const T*)L.x, (const T*)L.b,
                                 nullptr, (T)0, (T*)L.r, s);
  } else if (L.g.N <= p->small_nodes)
    launch_row_small<T>(L.g, opA<T>(L), opD<T>(L), (const T*)L.x, (const T*)L.b, (T*)L.r, (T)0, false, s);
  else
    launch_defect<T>(L.g, opA<T>(L), (const T*)L.x, (const T*)L.b, (T*)L.r, p->Cbuf, s, p->row_G[l]);
  if (l == 0 && p->timing)
    timer_end(p, p->t_resid,
              sizeof(T) * ((use_mf(p) ? 960.0 * L.g.NE : stored_blocks(L.g) * NBLK) + (double)L.g.N * 3 * NDOF));
  Level& C = p->lev[l + 1];
  launch_restrict<T>(L.g, C.g, (const T*)L.r, C.mask, (T*)C.b, s);
  vcycle<T>(p, l + 1);
  launch_prolong_add<T>(L.g, C.g, (const T*)C.x, L.mask, (T*)L.x, s);
  for (int k = 0; k < p->opts.nu_post; ++k) sweep<T>(p, l, false);
}

template <typename T, typename TZ>
void precondition(mvpf_problem* p, const double* v, TZ* z) {
  Level& L0 = p->lev[0];
  launch_convert_masked<double, T>(L0.g, v, L0.mask, (T*)L0.b, p->stream);
  vcycle<T>(p, 0);
  launch_precond_finish<T, TZ>(L0.g, (const T*)L0.x, v, L0.mask, z, p->stream);
}

// ---- FGMRES ---------------------------------------------------------------------
int fetch(mvpf_problem* p, const double* dsrc, int count) {
  HIPCHK(hipMemcpyAsync(p->hhost, dsrc, sizeof(double) * count, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int norm_device(mvpf_problem* p, int64_t n, const double* v, double* out_host) {
  const int nb = red_blocks(n);
  launch_multidot(n, v, n, 1, v, p->red, p->stream);
  launch_reduce(1, nb, p->red, p->hcol, 0, p->stream);
  TRY(launch_check(p, "norm"));
  TRY(fetch(p, p->hcol, 1));
  *out_host = std::sqrt(p->hhost[0]);
  return 0;
}

// Flexible GMRES(m), right preconditioned, x0 = 0, classical Gram-Schmidt
// twice, Givens rotations; convergence on the recurrence residual, then a
// true FP64 residual check (restart if it is not met).
//
// The iteration is a small state machine so that several problems can
// advance in lockstep with one host synchronisation per step (batched
// solves).  Each phase enqueues its device work on the problem's stream,
// ending with a copy of the scalars the host needs into pinned memory; the
// next phase runs on the host after the caller has synchronised.
//   ARNOLDI: the caller puts z_j = M^-1 v_j into zj(), then arnoldi_enqueue()
//            (outer product, CGS2, norm) ... sync ... arnoldi_finish()
//   CHECK:   (end of a cycle, work enqueued by arnoldi_finish) ... sync ...
//            check_finish(): converged, or restart (back to ARNOLDI)
template <typename T, typename TZ>
struct Krylov {
  enum Phase { START, ARNOLDI, CHECK, DONE };
  mvpf_problem* p = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  mvpf_solve_stats* st = nullptr;
  int64_t n = 0;
  int m = 0, nb = 0, j = 0, k = 0, rc = 0;
  Phase phase = START;
  // batched solves: the normalisation of the next basis vector is left to
  // the caller (pend_w *= pend_a), which batches it with other problems'
  bool defer = false;
  double* pend_w = nullptr;
  double pend_a = 0.0;
  std::vector<double> H, cs, sn, gg, y;
  double bnorm = 0.0, beta = 0.0;
  const double* r0 = nullptr;

  double& Hij(int i, int c) { return H[(size_t)i * m + c]; }
  double* h1() { return p->hcol; }
  double* h2() { return p->hcol + (MAX_RESTART + 2); }
  double* hn() { return p->hcol + 2 * (MAX_RESTART + 2); }
  double* vj() { return p->V + (int64_t)j * n; }
  TZ* zj() { return (TZ*)p->Z + (int64_t)j * n; }
  int fail(int code) {
    rc = code;
    phase = DONE;
    return code;
  }

  // zero x, ||b|| -> hhost[0]
  int begin(mvpf_problem* pp, const double* bb, double* xx, mvpf_solve_stats* ss) {
    p = pp;
    b = bb;
    x = xx;
    st = ss;
    n = nvec(p->lev[0].g);
    m = std::min(p->opts.restart, p->restart_cap);
    nb = red_blocks(n);
    H.assign((size_t)(m + 1) * m, 0.0);
    cs.assign(m, 0.0);
    sn.assign(m, 0.0);
    gg.assign(m + 1, 0.0);
    y.assign(m, 0.0);
    st->iterations = st->restarts = st->converged = 0;
    st->rel_residual = 0.0;
    hipStream_t s = p->stream;
    launch_zero<double>(n, x, s);
    launch_multidot(n, b, n, 1, b, p->red, s);
    launch_reduce(1, nb, p->red, p->hcol, 0, s);
    if (launch_check(p, "fgmres start") < 0) return fail(MVPF_EDEVICE);
    if (hipMemcpyAsync(p->hhost, p->hcol, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(MVPF_EDEVICE);
    phase = START;
    return 0;
  }
  void start_cycle() {
    launch_axpby(n, 1.0 / beta, r0, 0.0, nullptr, p->V, p->stream);
    std::fill(gg.begin(), gg.end(), 0.0);
    gg[0] = beta;
    j = 0;
    phase = ARNOLDI;
  }
  void after_begin() {
    bnorm = std::sqrt(p->hhost[0]);
    if (bnorm == 0.0) {
      st->converged = 1;
      phase = DONE;
      return;
    }
    beta = bnorm;
    r0 = b;
    start_cycle();
  }
  // w = A z_j, two Gram-Schmidt passes, ||w||^2; the three columns -> hhost
  int arnoldi_enqueue() {
    hipStream_t s = p->stream;
    const Grid& g = p->lev[0].g;
    double* w = p->V + (int64_t)(j + 1) * n;
    if (p->timing) timer_begin(p, p->t_outer);
    if (use_mf(p)) {
      mf_elements<double, TZ>(p, zj(), true);
      launch_mf_gather<0, double, TZ, double>(g, (const double*)p->Cbuf, contact(p), p->mf_epw, p->lev[0].mask, zj(),
                                              nullptr, nullptr, 0.0, w, s);
    } else {
      launch_spmv<double, TZ, double>(g, p->lev[0].A64, zj(), w, p->Cbuf, s, p->outer_G);
    }
    if (p->timing)
      timer_end(p, p->t_outer, 8.0 * (use_mf(p) ? 960.0 * g.NE : stored_blocks(g) * NBLK) +
                                   (double)g.N * NDOF * (sizeof(TZ) + sizeof(double)));
    launch_multidot(n, p->V, n, j + 1, w, p->red, s);
    launch_reduce(j + 1, nb, p->red, h1(), 0, s);
    launch_multiaxpy_dot(n, p->V, n, j + 1, h1(), w, p->red, s);
    launch_reduce(j + 1, nb, p->red, h2(), 0, s);
    launch_multiaxpy(n, p->V, n, j + 1, h2(), w, p->red, s);
    launch_reduce(1, nb, p->red, hn(), 0, s);
    if (launch_check(p, "fgmres arnoldi") < 0) return fail(MVPF_EDEVICE);
    if (hipMemcpyAsync(p->hhost, p->hcol, sizeof(double) * 3 * (MAX_RESTART + 2), hipMemcpyDeviceToHost, s) !=
        hipSuccess)
      return fail(MVPF_EDEVICE);
    return 0;
  }
  // Hessenberg column, Givens rotations; continue, or end the cycle
  int arnoldi_finish() {
    for (int i = 0; i <= j; ++i) Hij(i, j) = p->hhost[i] + p->hhost[(MAX_RESTART + 2) + i];
    const double hnext = std::sqrt(p->hhost[2 * (MAX_RESTART + 2)]);
    Hij(j + 1, j) = hnext;
    double* w = p->V + (int64_t)(j + 1) * n;
    if (hnext > 0.0) {
      if (defer) {
        pend_w = w;
        pend_a = 1.0 / hnext;
      } else {
        launch_axpby(n, 1.0 / hnext, w, 0.0, nullptr, w, p->stream);
      }
    }
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
      Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
      Hij(i, j) = t;
    }
    const double den = std::hypot(Hij(j, j), Hij(j + 1, j));
    cs[j] = Hij(j, j) / den;
    sn[j] = Hij(j + 1, j) / den;
    Hij(j, j) = den;
    Hij(j + 1, j) = 0.0;
    gg[j + 1] = -sn[j] * gg[j];
    gg[j] = cs[j] * gg[j];
    st->iterations++;
    k = j + 1;
    if (std::fabs(gg[j + 1]) <= p->opts.rtol * bnorm || st->iterations >= p->opts.max_it || k == m) {
      pend_w = nullptr;  // the cycle ends: v_{j+1} is not used
      return end_cycle_enqueue();
    }
    ++j;
    return 0;
  }
  // x += Z y, r = b - A x, ||r|| -> hhost[0]
  int end_cycle_enqueue() {
    hipStream_t s = p->stream;
    const Grid& g = p->lev[0].g;
    for (int i = k - 1; i >= 0; --i) {
      double sacc = gg[i];
      for (int c = i + 1; c < k; ++c) sacc -= Hij(i, c) * y[c];
      y[i] = sacc / Hij(i, i);
    }
    if (hipMemcpyAsync(h1(), y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(MVPF_EDEVICE);
    launch_combine<TZ>(n, (const TZ*)p->Z, n, k, h1(), x, s);
    if (use_mf(p)) {
      mf_elements<double, double>(p, x, true);
      launch_mf_gather<0, double, double, double>(g, (const double*)p->Cbuf, contact(p), p->mf_epw, p->lev[0].mask, x,
                                                  nullptr, nullptr, 0.0, p->tmp, s);
    } else {
      launch_spmv<double, double, double>(g, p->lev[0].A64, x, p->tmp, p->Cbuf, s, p->outer_G);
    }
    launch_axpby(n, 1.0, b, -1.0, p->tmp, p->tmp, s);
    launch_multidot(n, p->tmp, n, 1, p->tmp, p->red, s);
    launch_reduce(1, nb, p->red, p->hcol, 0, s);
    if (launch_check(p, "fgmres residual") < 0) return fail(MVPF_EDEVICE);
    if (hipMemcpyAsync(p->hhost, p->hcol, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(MVPF_EDEVICE);
    phase = CHECK;
    return 0;
  }
  void check_finish() {
    beta = std::sqrt(p->hhost[0]);
    st->rel_residual = beta / bnorm;
    if (st->rel_residual <= p->opts.rtol) {
      st->converged = 1;
      phase = DONE;
      return;
    }
    if (st->iterations >= p->opts.max_it) {
      rc = MVPF_ENOTCONV;
      phase = DONE;
      return;
    }
    st->restarts++;
    r0 = p->tmp;  // the next cycle overwrites V[0] from tmp before tmp is reused
    start_cycle();
  }
};

template <typename T, typename TZ>
int fgmres(mvpf_problem* p, const double* b, double* x, mvpf_solve_stats* st) {
  Krylov<T, TZ> K;
  TRY(K.begin(p, b, x, st));
  HIPCHK(hipStreamSynchronize(p->stream));
  K.after_begin();
  while (K.phase != Krylov<T, TZ>::DONE) {
    if (K.phase == Krylov<T, TZ>::ARNOLDI) {
      precondition<T, TZ>(p, K.vj(), K.zj());
      TRY(K.arnoldi_enqueue());
    }
    HIPCHK(hipStreamSynchronize(p->stream));
    if (K.phase == Krylov<T, TZ>::ARNOLDI)
      TRY(K.arnoldi_finish());
    else
      K.check_finish();
  }
  return K.rc;
}

int validate(const mvpf_mesh* mesh, const mvpf_material* mat, const mvpf_loading* load, const mvpf_opts* o,
             std::string& err) {
  if (!mesh || !mat || !load || !o) { err = "null argument"; return MVPF_EINVAL; }
  if (mesh->nx < 2 || mesh->ny < 2 || mesh->nz < 2 || !(mesh->h > 0)) { err = "bad mesh sizes"; return MVPF_EINVAL; }
  if (mesh->n_levels < 2 || mesh->n_levels > MAX_LEVELS) { err = "n_levels must be in [2, 8]"; return MVPF_EINVAL; }
  const int f = 1 << (mesh->n_levels - 1);
  if (mesh->nx % f || mesh->ny % f || mesh->nz % f) {
    err = "nx, ny, nz must be divisible by 2^(n_levels-1)";
    return MVPF_EINVAL;
  }
  const int64_t nc = (int64_t)(mesh->nx / f + 1) * (mesh->ny / f + 1) * (mesh->nz / f + 1) * NDOF;
  if (nc > MVPF_MAX_COARSE_DOF) { err = "coarsest level too large for the dense direct solve"; return MVPF_EINVAL; }
  const int64_t nn = (int64_t)(mesh->nx + 1) * (mesh->ny + 1) * (mesh->nz + 1);
  if (nn * NDOF * 27 * 9 > ((int64_t)1 << 62) || nn >= ((int64_t)1 << 31) - 64) {
    err = "mesh too large";
    return MVPF_EINVAL;
  }
  if (mat->pade != 11 && mat->pade != 22 && mat->pade != 33) {
    err = "Pade order of the Hencky strain must be 11, 22 or 33";
    return MVPF_EINVAL;
  }
  if (mat->mixing != MVPF_MIX_LINEAR && mat->mixing != MVPF_MIX_LOG) {
    err = "mixing must be MVPF_MIX_LINEAR or MVPF_MIX_LOG";
    return MVPF_EINVAL;
  }
  if (load->kind == MVPF_LOAD_PATCH) {
    if (load->patch < 0 || load->patch % 2 || mesh->nx % 2 || mesh->ny % 2) {
      err = "patch loading needs even patch, nx and ny";
      return MVPF_EINVAL;
    }
  } else if (load->kind == MVPF_LOAD_CAP) {
    if (!(load->radius > 0)) { err = "cap radius must be positive"; return MVPF_EINVAL; }
  } else if (load->kind == MVPF_LOAD_SPHERE) {
    if (!(load->radius > 0) || !(load->eps_n > 0)) {
      err = "sphere contact needs a positive radius and eps_n";
      return MVPF_EINVAL;
    }
  } else {
    err = "unknown loading kind";
    return MVPF_EINVAL;
  }
  if (o->precision != MVPF_FP64 && o->precision != MVPF_MIXED) { err = "bad precision"; return MVPF_EINVAL; }
  if (o->restart < 1 || o->restart > MAX_RESTART || o->max_it < 1 || !(o->rtol > 0)) {
    err = "bad Krylov options";
    return MVPF_EINVAL;
  }
  if (o->nu_pre < 0 || o->nu_post < 0 || !(o->omega > 0) || o->newton_max < 1) {
    err = "bad smoother/Newton options";
    return MVPF_EINVAL;
  }
  if (o->coarse != MVPF_COARSE_REDISCRETISE && o->coarse != MVPF_COARSE_GALERKIN) {
    err = "coarse must be MVPF_COARSE_REDISCRETISE or MVPF_COARSE_GALERKIN";
    return MVPF_EINVAL;
  }
  return 0;
}

void destroy_all(mvpf_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (int l = 0; l < MAX_LEVELS; ++l) {
    Level& L = p->lev[l];
    dfree(L.state); dfree(L.mask); dfree(L.target); dfree(L.A64); dfree(L.A32); dfree(L.diag64);
    dfree(L.Dinv64); dfree(L.Dinv32); dfree(L.DinvS32);
    dfree(L.x); dfree(L.x2); dfree(L.b); dfree(L.r); dfree(L.Ainv);
  }
  for (int l = 0; l < MAX_LEVELS; ++l) dfree(p->gal[l]);
  dfree(p->Dmf64); dfree(p->Dmf32); dfree(p->sphere);
  dfree(p->card); dfree(p->qp); dfree(p->elem); dfree(p->Cbuf); dfree(p->R); dfree(p->rhs); dfree(p->gvec); dfree(p->dx); dfree(p->tmp);
  dfree(p->tmp2); dfree(p->V); dfree(p->Z); dfree(p->red); dfree(p->hcol); dfree(p->save_state);
  if (p->side) (void)hipStreamSynchronize(p->side);
  dfree(p->coarse_work);
  if (p->hhost) (void)hipHostFree(p->hhost);
  p->hhost = nullptr;
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->side) (void)hipStreamDestroy(p->side);
  p->ev_fork = p->ev_join = nullptr;
  p->side = nullptr;
  for (KernelTimer* t : {&p->t_sweep, &p->t_outer, &p->t_resid, &p->t_qp})
    for (hipEvent_t e : t->ev) (void)hipEventDestroy(e);
}

int allocate(mvpf_problem* p) {
  const mvpf_mesh& M = p->mesh;
  p->L = M.n_levels;
  p->mixed = p->opts.precision == MVPF_MIXED;
  p->mf = p->mf && p->L > 1;  // a one-level problem is solved densely
  for (int l = 0; l < p->L; ++l) {
    const int f = 1 << l;
    Level& L = p->lev[l];
    L.g = make_grid(M.nx / f, M.ny / f, M.nz / f, M.h * f);
    const bool coarsest = (l == p->L - 1);
    const int64_t nv = nvec(L.g);
    const int64_t nA64 = (int64_t)L.g.ntiles * NUP * Lay<double>::SLICE;
    const int64_t nA32 = (int64_t)L.g.ntiles * NUP * Lay<float>::SLICE;
    const int64_t nD64 = (int64_t)L.g.ntiles * Lay<double>::SLICE;
    const int64_t nD32 = (int64_t)L.g.ntiles * Lay<float>::SLICE;
    TRY(dalloc(p, &L.state, (size_t)NSTATE * L.g.Npad));
    TRY(dalloc(p, &L.mask, (size_t)L.g.Npad));
    if (l == 0) TRY(dalloc(p, &L.target, (size_t)L.g.Npad));
    const bool mf0 = l == 0 && p->mf;  // matrix-free finest level: no stored blocks
    if (!mf0 && (l == 0 || !p->mixed || coarsest)) TRY(dalloc(p, &L.A64, (size_t)nA64));
    if (!mf0 && p->mixed && !coarsest) TRY(dalloc(p, &L.A32, (size_t)nA32));
    if (mf0) {
      TRY(dalloc(p, &p->Dmf64, mf_hessian_values(L.g)));
      if (p->mixed) TRY(dalloc(p, &p->Dmf32, mf_hessian_values(L.g)));
    }
    if (!coarsest) {
      TRY(dalloc(p, &L.diag64, (size_t)nD64));
      if (p->mixed)
        TRY(dalloc(p, &L.Dinv32, (size_t)nD32));
      else
        TRY(dalloc(p, &L.Dinv64, (size_t)nD64));
      if (mf0 && p->mixed) TRY(dalloc(p, &L.DinvS32, (size_t)L.g.ntiles * LaySym<float>::SLICE));
    }
    const size_t es = p->mixed ? sizeof(float) : sizeof(double);
    for (void** v : {&L.x, &L.x2, &L.b, &L.r}) {
      char* c = nullptr;
      TRY(dalloc(p, &c, (size_t)nv * es));
      *v = c;
    }
    if (coarsest) {
      L.ndense = NDOF * L.g.N;
      TRY(dalloc(p, &L.Ainv, (size_t)L.ndense * L.ndense));
    }
  }
  const Grid& g0 = p->lev[0].g;
  const int64_t n = nvec(g0);
  TRY(dalloc(p, &p->card, 1));
  if (p->load.kind == MVPF_LOAD_SPHERE) TRY(dalloc(p, &p->sphere, 1));
  {
    // Gauss-point and element-matrix buffers: the whole finest level if that
    // fits ASSEMBLY_FULL_MAX bytes, else slabs of ASSEMBLY_SLAB_BYTES
    const int64_t per = (int64_t)(QP_HESS_ALLOC * 8 + NPAIR * NBLK) * (int64_t)sizeof(double);
    const int64_t nxy = (int64_t)g0.nx * g0.ny;
    if ((int64_t)g0.NEpad * per <= ASSEMBLY_FULL_MAX)
      p->ne_cap = g0.NEpad;
    else
      p->ne_cap = std::max<int64_t>(ASSEMBLY_SLAB_BYTES / per, 2 * nxy + TILE) / TILE * TILE;
    p->ne_cap = std::min<int64_t>(p->ne_cap, g0.NEpad);
    p->ne_use = p->ne_cap;
    TRY(dalloc(p, &p->qp, (size_t)QP_HESS_ALLOC * 8 * p->ne_cap));
    TRY(dalloc(p, &p->elem, (size_t)NPAIR * NBLK * p->ne_cap));
  }
  {
    // transposed half-stencil contributions, or the matrix-free element outputs
    double* cb = nullptr;
    TRY(dalloc(p, &cb, (size_t)std::max<int64_t>((int64_t)(NUP - 1) * NDOF * g0.Npad, mf_out_values(g0))));
    p->Cbuf = cb;
  }
  for (double** v : {&p->R, &p->rhs, &p->gvec, &p->dx, &p->tmp, &p->tmp2}) TRY(dalloc(p, v, (size_t)n));
  p->restart_cap = p->opts.restart;
  TRY(dalloc(p, &p->V, (size_t)(p->restart_cap + 1) * n));
  {
    char* z = nullptr;
    TRY(dalloc(p, &z, (size_t)p->restart_cap * n * (p->mixed ? sizeof(float) : sizeof(double))));
    p->Z = z;
  }
  TRY(dalloc(p, &p->red, (size_t)(MAX_RESTART + 2) * MAX_RED_BLOCKS));
  TRY(dalloc(p, &p->hcol, (size_t)3 * (MAX_RESTART + 2)));
  TRY(dalloc(p, &p->save_state, (size_t)NSTATE * g0.Npad));
  // Krylov scalars (3 columns) + one slot for the setup status
  hipError_t e = hipHostMalloc((void**)&p->hhost, sizeof(double) * (3 * (MAX_RESTART + 2) + 1));
  if (e != hipSuccess) {
    p->err = "hipHostMalloc failed";
    return MVPF_ENOMEM;
  }
  HIPCHK(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  {
    // dense coarse operator + inversion workspace; reuses the Krylov basis V
    // (idle during assembly) when it is large enough
    const int nd = p->lev[p->L - 1].ndense;
    const int64_t need = (int64_t)nd * nd + (int64_t)(dense_invert_work(nd) / sizeof(double)) + 1;
    const int64_t have = (int64_t)(p->restart_cap + 1) * n;
    if (need > have) TRY(dalloc(p, &p->coarse_work, (size_t)need));
  }
  DevCard hc;
  make_card(p, hc);
  p->pade = hc.pade;
  p->mixing = hc.mixing;
  HIPCHK(hipMemcpyAsync(p->card, &hc, sizeof(DevCard), hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int free_norm(mvpf_problem* p, const double* v, double* out) {
  const Grid& g = p->lev[0].g;
  const int nb = red_blocks((int64_t)g.N * NDOF);
  launch_free_norm_partial(g, v, p->lev[0].mask, p->red, p->stream);
  launch_reduce(1, nb, p->red, p->hcol, 0, p->stream);
  TRY(launch_check(p, "free norm"));
  TRY(fetch(p, p->hcol, 1));
  *out = std::sqrt(p->hhost[0]);
  return 0;
}

// residual at the current state into p->R (masks of `depth` for the norm)
bool contact(const mvpf_problem* p) { return p->load.kind == MVPF_LOAD_SPHERE; }

int compute_residual(mvpf_problem* p, double depth, double* norm_free) {
  Level& L0 = p->lev[0];
  launch_dirichlet_masks(L0.g, p->load, depth, L0.mask, L0.target, p->stream);
  for (const Chunk& ck : make_chunks(L0.g, p->ne_use)) {
    launch_qp(L0.g, ck, L0.state, p->card, p->pade, p->mixing, p->qp, false, p->stream);
    launch_residual_gather(L0.g, ck, L0.state, p->qp, p->card, p->R, p->stream);
  }
  if (contact(p)) launch_contact_residual(L0.g, make_sphere(L0.g, p->load, depth), L0.state, p->R, p->stream);
  TRY(launch_check(p, "residual"));
  if (norm_free) TRY(free_norm(p, p->R, norm_free));
  return 0;
}

// reassembly of level l >= 1 at its injected state (Sec. 3.4: rediscretised
// coarse operators, contact included); the state must already be injected
void assemble_coarse_level(mvpf_problem* p, int l, double depth) {
  Level& C = p->lev[l];
  for (const Chunk& ck : make_chunks(C.g, p->ne_use)) {
    launch_qp(C.g, ck, C.state, p->card, p->pade, p->mixing, p->qp, true, p->stream);
    launch_element_matrices(C.g, ck, p->qp, p->card, p->elem, p->stream);
    if (contact(p)) launch_contact_element(C.g, ck, make_sphere(C.g, p->load, depth), C.state, p->elem, p->stream);
    launch_jacobian_gather(C.g, ck, p->elem, C.A64, C.A32, C.diag64, p->stream);
  }
  launch_apply_dirichlet(C.g, C.mask, C.A64, C.A32, C.diag64, p->stream);
}

int* setup_status(mvpf_problem* p) { return (int*)p->red; }  // first word of the reduction scratch

// The coarsest operator is assembled first; its dense gather and inversion
// then run on the side stream while the main stream assembles the finer
// levels.  setup_solver joins the two streams.
// coarse_inline = false (batches): the coarsest operator is gathered into its
// dense matrix on the problem's stream, ev_fork marks it ready, and the
// batch inverts all problems' matrices at once and records ev_join.
// status word, Dirichlet masks of `depth`, injected masks and states
int system_prelude(mvpf_problem* p, double depth) {
  hipStream_t s = p->stream;
  Level& L0 = p->lev[0];
  HIPCHK(hipMemsetAsync(setup_status(p), 0, sizeof(int), s));
  launch_dirichlet_masks(L0.g, p->load, depth, L0.mask, L0.target, s);
  for (int l = 1; l < p->L; ++l) {
    launch_inject_mask(p->lev[l - 1].g, p->lev[l].g, p->lev[l - 1].mask, p->lev[l].mask, s);
    launch_inject(p->lev[l - 1].g, p->lev[l].g, p->lev[l - 1].state, p->lev[l].state, s);
  }
  return 0;
}

// after the finest tangent: contact residual, lifting of the prescribed
// increment and the right-hand side (the symmetric elimination follows)
int system_rhs(mvpf_problem* p, double depth) {
  hipStream_t s = p->stream;
  Level& L0 = p->lev[0];
  if (contact(p)) {
    launch_contact_residual(L0.g, make_sphere(L0.g, p->load, depth), L0.state, p->R, s);
    const Sphere sp = make_sphere(L0.g, p->load, depth);
    HIPCHK(hipMemcpyAsync(p->sphere, &sp, sizeof(Sphere), hipMemcpyHostToDevice, s));
  }
  launch_increment(L0.g, L0.mask, L0.target, L0.state, p->gvec, s);
  if (use_mf(p)) {
    mf_elements<double, double>(p, p->gvec, false, true);
    launch_mf_gather<0, double, double, double>(L0.g, (const double*)p->Cbuf, contact(p), p->mf_epw, nullptr, p->gvec,
                                                nullptr, nullptr, 0.0, p->tmp, s);
  } else {
    launch_spmv<double, double, double>(L0.g, L0.A64, p->gvec, p->tmp, p->Cbuf, s);
  }
  launch_newton_rhs(L0.g, L0.mask, p->R, p->tmp, p->gvec, p->rhs, s);
  return 0;
}

double* coarse_dense(mvpf_problem* p) { return p->coarse_work ? p->coarse_work : p->V; }

// the coarsest level's eliminated operator -> dense matrix; marks it ready
int coarse_fork(mvpf_problem* p, bool coarse_inline) {
  Level& C = p->lev[p->L - 1];
  launch_dense_from_bsr(C.g, C.A64, coarse_dense(p), p->stream);
  HIPCHK(hipEventRecord(p->ev_fork, p->stream));
  if (!coarse_inline) p->coarse_pending = true;
  return 0;
}

// the smoother's block inverses, enqueued before the coarse inversion's long
// chain of launches (the host can block while it enqueues that chain), then
// the inversion (on the side stream when it overlaps)
int finish_system(mvpf_problem* p, bool coarse_inline) {
  hipStream_t s = p->stream;
  for (int l = 0; l < p->L - 1; ++l) {
    Level& L = p->lev[l];
    launch_block_inverse(L.g, L.diag64, L.Dinv64, L.Dinv32, L.DinvS32, setup_status(p), s);
  }
  TRY(launch_check(p, "assembly"));
  if (coarse_inline) {
    Level& C = p->lev[p->L - 1];
    const int nd = C.ndense;
    double* work = coarse_dense(p);
    const bool overlap = p->coarse_overlap < 0 ? nd <= COARSE_OVERLAP_MAX : p->coarse_overlap != 0;
    hipStream_t cs = overlap ? p->side : s;
    if (overlap) HIPCHK(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    if (dense_invert(nd, work, C.Ainv, work + (int64_t)nd * nd, setup_status(p), cs) != 0) {
      p->err = "coarse inversion launch failed";
      return MVPF_EDEVICE;
    }
    if (overlap) {
      HIPCHK(hipEventRecord(p->ev_join, p->side));
      p->coarse_pending = true;
    }
    TRY(launch_check(p, "coarse inversion"));
  }
  return 0;
}

// Galerkin hierarchy (opts.coarse = MVPF_COARSE_GALERKIN, galerkin.hip): the
// finest tangent's element matrices (all 36 node pairs, contact included)
// are coarsened slab by slab into level 1's, each level's into the next's;
// every coarse level's stored blocks are gathered from its element matrices.
// The coarsest level is finished first so that its inversion overlaps the
// intermediate levels' gathers and the block inverses.
int build_system_galerkin(mvpf_problem* p, double depth, bool coarse_inline) {
  hipStream_t s = p->stream;
  Level& L0 = p->lev[0];
  const int Lc = p->L - 1;
  for (int l = 1; l < p->L; ++l)
    if (!p->gal[l]) TRY(dalloc(p, &p->gal[l], (size_t)NPAIR * NBLK * p->lev[l].g.NEpad));
  TRY(system_prelude(p, depth));
  const bool mf = use_mf(p);
  const Grid& g1 = p->lev[1].g;
  const int64_t nxy = (int64_t)L0.g.nx * L0.g.ny;
  int zdone = 0;  // level-1 element layers coarsened so far
  for (const Chunk& ck : make_chunks(L0.g, p->ne_use)) {
    timer_begin(p, p->t_qp);
    launch_qp(L0.g, ck, L0.state, p->card, p->pade, p->mixing, p->qp, true, s);
    timer_end(p, p->t_qp, 8.0 * 8 * QP_HESS * (double)ck.NEc);
    if (mf) launch_mf_pack(L0.g, ck, p->qp, p->Dmf64, p->Dmf32, s);
    launch_residual_gather(L0.g, ck, L0.state, p->qp, p->card, p->R, s);
    launch_element_matrices(L0.g, ck, p->qp, p->card, p->elem, s, false);
    if (contact(p)) launch_contact_element(L0.g, ck, make_sphere(L0.g, p->load, depth), L0.state, p->elem, s, false);
    launch_jacobian_gather(L0.g, ck, p->elem, L0.A64, L0.A32, L0.diag64, s, mf);
    // level-1 layers Z whose child layers 2Z and 2Z + 1 this slab holds (slabs
    // overlap by one element layer, so each layer is met in one of them)
    const int ez0 = (int)(ck.e0 / nxy), ez1 = (int)((ck.e0 + ck.NEc) / nxy);
    const int z1 = ez1 / 2;
    if (zdone < z1) {
      if (2 * zdone < ez0) {
        p->err = "internal: an assembly slab does not hold the child layers of a coarse layer";
        return MVPF_EDEVICE;
      }
      launch_galerkin_coarsen(L0.g, ck, p->elem, L0.mask, g1, zdone, z1, p->gal[1], s);
      zdone = z1;
    }
  }
  if (zdone != g1.nz) {
    p->err = "internal: coarse layers left out of the Galerkin product";
    return MVPF_EDEVICE;
  }
  TRY(system_rhs(p, depth));
  launch_apply_dirichlet(L0.g, L0.mask, L0.A64, L0.A32, L0.diag64, s);
  auto whole = [](const Grid& g) { return Chunk{0, g.NE, g.NEpad, 0, g.Npad}; };
  for (int l = 1; l < Lc; ++l) {
    const Grid& g = p->lev[l].g;
    launch_galerkin_coarsen(g, whole(g), p->gal[l], p->lev[l].mask, p->lev[l + 1].g, 0, p->lev[l + 1].g.nz,
                            p->gal[l + 1], s);
  }
  for (int l = Lc; l >= 1; --l) {
    Level& C = p->lev[l];
    launch_jacobian_gather(C.g, whole(C.g), p->gal[l], C.A64, C.A32, C.diag64, s);
    launch_apply_dirichlet(C.g, C.mask, C.A64, C.A32, C.diag64, s);
    if (l == Lc) TRY(coarse_fork(p, coarse_inline));
  }
  return finish_system(p, coarse_inline);
}

int build_system(mvpf_problem* p, double depth, bool coarse_inline = true) {
  if (p->opts.coarse == MVPF_COARSE_GALERKIN) return build_system_galerkin(p, depth, coarse_inline);
  hipStream_t s = p->stream;
  Level& L0 = p->lev[0];
  const int Lc = p->L - 1;
  TRY(system_prelude(p, depth));
  // coarsest level first, as a dense matrix; its inversion (a chain of
  // several hundred launches) is enqueued after the finer levels' assembly,
  // so that the host feeds the main stream first and the side stream's chain
  // then runs beside it
  assemble_coarse_level(p, Lc, depth);
  TRY(launch_check(p, "coarse assembly"));
  TRY(coarse_fork(p, coarse_inline));
  for (int l = Lc - 1; l >= 1; --l) assemble_coarse_level(p, l, depth);
  // finest: residual and unconstrained tangent
  for (const Chunk& ck : make_chunks(L0.g, p->ne_use)) {
    timer_begin(p, p->t_qp);
    launch_qp(L0.g, ck, L0.state, p->card, p->pade, p->mixing, p->qp, true, s);
    // written: gradient (15) and packed Hessian (120) per Gauss point
    timer_end(p, p->t_qp, 8.0 * 8 * QP_HESS * (double)ck.NEc);
    const bool mf = use_mf(p);  // only the diagonal blocks are assembled
    if (mf) launch_mf_pack(L0.g, ck, p->qp, p->Dmf64, p->Dmf32, s);
    launch_residual_gather(L0.g, ck, L0.state, p->qp, p->card, p->R, s);
    launch_element_matrices(L0.g, ck, p->qp, p->card, p->elem, s, mf);
    if (contact(p)) launch_contact_element(L0.g, ck, make_sphere(L0.g, p->load, depth), L0.state, p->elem, s, mf);
    launch_jacobian_gather(L0.g, ck, p->elem, L0.A64, L0.A32, L0.diag64, s, mf);
  }
  // lifting of the prescribed increment, then symmetric elimination
  TRY(system_rhs(p, depth));
  launch_apply_dirichlet(L0.g, L0.mask, L0.A64, L0.A32, L0.diag64, s);
  return finish_system(p, coarse_inline);
}

// pinned host slot of the setup status
int* host_status(mvpf_problem* p) { return (int*)(p->hhost + 3 * (MAX_RESTART + 2)); }

// joins the coarse inversion; status -> host (build_system enqueued the
// smoother's block inverses)
int setup_enqueue(mvpf_problem* p) {
  hipStream_t s = p->stream;
  int* status = setup_status(p);
  if (p->coarse_pending) {
    HIPCHK(hipStreamWaitEvent(s, p->ev_join, 0));
    p->coarse_pending = false;
  }
  TRY(launch_check(p, "solver setup"));
  HIPCHK(hipMemcpyAsync(host_status(p), status, sizeof(int), hipMemcpyDeviceToHost, s));
  return 0;
}

// after the problem's stream has been synchronised
int setup_finish(mvpf_problem* p) {
  if (*host_status(p)) {
    p->err = "singular 9x9 diagonal block or coarse operator";
    return MVPF_ESINGULAR;
  }
  return 0;
}

int setup_solver(mvpf_problem* p) {
  TRY(setup_enqueue(p));
  HIPCHK(hipStreamSynchronize(p->stream));
  return setup_finish(p);
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

int solve_internal(mvpf_problem* p, const double* b, double* x, mvpf_solve_stats* st) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, p->stream));
  int rc = p->mixed ? fgmres<float, float>(p, b, x, st) : fgmres<double, double>(p, b, x, st);
  (void)hipEventRecord(e1, p->stream);
  (void)hipEventSynchronize(e1);
  st->solve_ms = elapsed_ms(e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

namespace {
// time `reps` launches of f on the problem's stream (ms per launch)
template <typename Fn>
double time_launches(mvpf_problem* p, int reps, Fn f) {
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  f();  // warm-up
  (void)hipEventRecord(a, p->stream);
  for (int i = 0; i < reps; ++i) f();
  (void)hipEventRecord(b, p->stream);
  (void)hipEventSynchronize(b);
  const double ms = elapsed_ms(a, b) / reps;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

// Candidate persistent launch shapes for a level: fixed sizes, plus the
// divisors of the row-block count that give every workgroup the same number
// of blocks in one residency round (no partial last wave).
std::vector<int> launch_candidates(const Grid& g) {
  std::vector<int> c = {0, 4096, 2048, 1536, 1024, 768, 512, 384, 256, 192, 128, 96, 64};
  const int nb = (g.Npad + 255) / 256;
  for (int k = 2; k <= 4; ++k) c.push_back(((nb + k - 1) / k + 7) / 8 * 8);
  return c;
}

// Tuning results, reused by later problems of the same shape: keyed by the
// GPU architecture, the multigrid precision, the finest-level mode, the
// tuned quantity and the level's element counts.  Process-wide; when the
// environment variable MVPF_TUNE_CACHE names a file, entries are read from it
// once and every new entry is appended to it ("key value" lines).
struct TuneCache {
  std::mutex mu;
  std::map<std::string, int> entries;
  bool loaded = false;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}
std::string tune_key(const mvpf_problem* p, const char* what, const Grid& g) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  const std::string::size_type c = arch.find(':');
  if (c != std::string::npos) arch.resize(c);
  return arch + "/" + (p->mixed ? "mixed" : "fp64") + "/" + (use_mf(p) ? "mf" : "asm") + "/" + what + "/" +
         std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" + std::to_string(g.nz);
}
bool tune_lookup(const std::string& key, int* value) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  if (!c.loaded) {
    c.loaded = true;
    if (const char* path = std::getenv("MVPF_TUNE_CACHE")) {
      std::ifstream in(path);
      std::string k;
      int v;
      while (in >> k >> v) c.entries[k] = v;
    }
  }
  auto it = c.entries.find(key);
  if (it == c.entries.end()) return false;
  *value = it->second;
  return true;
}
void tune_store(const std::string& key, int value) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  c.entries[key] = value;
  if (const char* path = std::getenv("MVPF_TUNE_CACHE")) {
    std::ofstream out(path, std::ios::app);
    out << key << " " << value << "\n";
  }
}

template <typename T>
void autotune_levels(mvpf_problem* p, int* tuned) {
  const bool cached = p->tune_cache_use != 0;
  int hit = 0;
  if (use_mf(p) && cached && tune_lookup(tune_key(p, "mf_epw", p->lev[0].g), &hit)) {
    p->mf_epw = hit;
    tuned[0] = hit;
  } else if (use_mf(p)) {  // elements per workgroup of the matrix-free smoother sweep
    Level& L = p->lev[0];
    double best = 1e30;
    int bestE = 32;
    for (int epw : {32, 16, 8}) {
      p->mf_epw = epw;
      const double ms = time_launches(p, 5, [&] {
        mf_elements<T, T>(p, (const T*)L.x, true);
        launch_mf_gather<2, T, T, T>(L.g, (const T*)p->Cbuf, contact(p), p->mf_epw, L.mask, (const T*)L.x,
                                     (const T*)L.b, mfDinv<T>(L), (T)p->opts.omega, (T*)L.x2, p->stream);
      });
      if (ms < best * 0.98) { best = ms; bestE = epw; }
    }
    p->mf_epw = bestE;
    tuned[0] = bestE;
    tune_store(tune_key(p, "mf_epw", L.g), bestE);
  }
  for (int l = 0; l < p->L - 1; ++l) {
    Level& L = p->lev[l];
    if (L.g.N <= p->small_nodes) continue;  // small-grid kernels have a fixed shape
    if (l == 0 && use_mf(p)) continue;      // tuned above
    if (cached && tune_lookup(tune_key(p, "row_blocks", L.g), &hit)) {
      p->row_G[l] = hit;
      tuned[l] = hit;
      continue;
    }
    double best = 1e30;
    int bestG = 0;
    for (int G : launch_candidates(L.g)) {
      const double ms = time_launches(p, 5, [&] {
        launch_pbj<T>(L.g, opA<T>(L), opD<T>(L), (const T*)L.x, (const T*)L.b, (T*)L.x2, (T)p->opts.omega, false,
                      p->Cbuf, p->stream, G);
      });
      if (ms < best * 0.98) { best = ms; bestG = G; }
    }
    p->row_G[l] = bestG;
    tuned[l] = bestG;
    tune_store(tune_key(p, "row_blocks", L.g), bestG);
  }
  const Grid& g = p->lev[0].g;
  if (use_mf(p)) return;
  if (cached && tune_lookup(tune_key(p, "outer_blocks", g), &hit)) {
    p->outer_G = hit;
    tuned[p->L - 1] = hit;
    return;
  }
  double best = 1e30;
  int bestG = 0;
  for (int G : launch_candidates(g)) {
    const double ms = time_launches(p, 5, [&] {
      if (p->mixed)
        launch_spmv<double, float, double>(g, p->lev[0].A64, (const float*)p->Z, p->tmp, p->Cbuf, p->stream, G);
      else
        launch_spmv<double, double, double>(g, p->lev[0].A64, p->tmp2, p->tmp, p->Cbuf, p->stream, G);
    });
    if (ms < best * 0.98) { best = ms; bestG = G; }
  }
  p->outer_G = bestG;
  tuned[p->L - 1] = bestG;
  tune_store(tune_key(p, "outer_blocks", g), bestG);
}
}  // namespace

// =============================================================================
// Batches of independent problems
// =============================================================================
// HIPCHK for batch-level code (error text goes to the batch)
#define BCHK(call)                                                               \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      b->err = std::string(#call) + " failed: " + hipGetErrorString(e_);         \
      return MVPF_EDEVICE;                                                       \
    }                                                                            \
  } while (0)

struct mvpf_batch {
  int n = 0;
  bool mixed = false;
  hipStream_t stream = nullptr;
  std::vector<mvpf_problem*> probs;
  // inputs and outputs of the V-cycle graph for problems not in an Arnoldi
  // step (FP64 in, FP32 out in mixed mode); the others read v_j, write z_j
  std::vector<double*> vin;
  std::vector<void*> zout;
  // per-problem streams (the assembly stream of batched systems is branch[0];
  // systems with slabs assemble each problem on its own stream)
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  // the batched solve runs on its own stream (graphs cannot be captured on
  // the legacy default stream), ordered after and before the caller's stream
  hipStream_t work = nullptr;
  hipEvent_t enter = nullptr, leave = nullptr;
  // the coarsest-level inversions of all problems as one batched inversion
  mvpf::GJJob* gj_tab = nullptr;
  int* gj_sel = nullptr;
  std::vector<int> gj_n;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> graph_version;  // config_version of each problem at capture
  // job tables of the graph's batched launches (device); the preconditioner's
  // ends (input v_j, output z_j of each problem) are rewritten every step
  mvpf::BJob* jobs_dev = nullptr;
  size_t jobs_cap = 0;
  size_t conv_off = 0, fin_off = 0;
  std::vector<mvpf::BJob> conv_jobs, fin_jobs;
  // per-step job tables of the batched Arnoldi step (pinned host staging and
  // device copies) and the Hessenberg columns of all problems
  mvpf::KJob *kjobs_host = nullptr, *kjobs_dev = nullptr;
  // job table of the batched assembly (device)
  mvpf::AJob* ajobs_dev = nullptr;
  size_t ajobs_cap = 0;
  mvpf::BJob *ojobs_host = nullptr, *ojobs_dev = nullptr, *gjobs_host = nullptr;
  double *bcol_dev = nullptr, *bcol_host = nullptr;
  std::string err;
};

namespace {

void batch_drop_graph(mvpf_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// ---- the batched V-cycle: one launch per operator for all problems ----------
// The V-cycles of all problems are laid out as one sequence of batched
// launches.  At every step of the cycle the problems are grouped by kernel
// family (matrix-free finest level, two-pass half-stencil, small grid), each
// group being one launch whose jobs are the problems of the group; every
// problem sees exactly the kernels and summation orders of its own V-cycle,
// so its result is bitwise that of preconditioning it alone.  The few
// per-problem launches left (contact stiffness, a zero first guess without
// pre-smoothing) are kept as such.
struct PlanOp {
  int op = -1;  // BatchOp, or -1 for a per-problem launch
  std::vector<BJob> jobs;
  size_t off = 0;
  int blocks = 0;
  int threads = 256;  // workgroup size of the matrix-free element kernels
  std::function<void(hipStream_t)> solo;
};

struct Planner {
  std::vector<PlanOp> ops;
  // one launch per op kind: jobs[k] go into a new op of kind kinds[k]
  void add(int op, std::vector<BJob>&& jobs, int threads = 256) {
    if (jobs.empty()) return;
    PlanOp o;
    o.op = op;
    o.jobs = std::move(jobs);
    o.threads = threads;
    ops.push_back(std::move(o));
  }
  void solo(std::function<void(hipStream_t)> f) {
    PlanOp o;
    o.solo = std::move(f);
    ops.push_back(std::move(o));
  }
};

BJob job_of(const Level& L) {
  BJob j{};
  j.g = L.g;
  j.mask = L.mask;
  return j;
}

// Elements per workgroup of a batched matrix-free element launch: the tuned
// value of its largest problem (results do not depend on it).
int batch_mf_epw(const std::vector<mvpf_problem*>& ps) {
  int epw = 32;
  int64_t most = -1;
  for (const mvpf_problem* p : ps)
    if (p->lev[0].g.NE > most) {
      most = p->lev[0].g.NE;
      epw = p->mf_epw;
    }
  return mf_epw_of(epw);
}
// the gathers of a batched matrix-free product read what the element launch
// of batch_mf_epw(mf) wrote, contact face outputs included
void set_mf_gathers(std::vector<BJob>& gather, const std::vector<mvpf_problem*>& mf) {
  const int epw = batch_mf_epw(mf);
  for (size_t i = 0; i < gather.size(); ++i) {
    gather[i].epw = epw;
    gather[i].contact = contact(mf[i]);
  }
}

template <typename T>
void plan_mf_elements(Planner& pl, const std::vector<mvpf_problem*>& mf) {
  std::vector<BJob> el;
  for (mvpf_problem* p : mf) {
    Level& L = p->lev[0];
    BJob j = job_of(L);
    j.A = mfD<T>(p);
    j.x = L.x;
    j.cd = p->card;
    j.C = p->Cbuf;
    el.push_back(j);
  }
  pl.add(BOP_MF_ELEMENT, std::move(el), 8 * batch_mf_epw(mf));
  for (mvpf_problem* p : mf)
    if (contact(p)) {
      Level& L = p->lev[0];
      const T* x = (const T*)L.x;
      pl.solo([p, x](hipStream_t s) {
        Level& L0 = p->lev[0];
        launch_contact_apply<T, T>(L0.g, p->sphere, L0.state, L0.mask, x, (T*)p->Cbuf, s);
      });
    }
}

// damped point-block Jacobi sweeps on level l of every problem in ps
template <typename T>
void plan_sweep(Planner& pl, const std::vector<mvpf_problem*>& ps, int l, bool zero) {
  std::vector<mvpf_problem*> mf;
  std::vector<BJob> z, split, lower, small, gather;
  for (mvpf_problem* p : ps) {
    Level& L = p->lev[l];
    BJob j = job_of(L);
    j.omega = p->opts.omega;
    j.D = opD<T>(L);
    j.x = L.x;
    j.b = L.b;
    j.y = L.x2;
    if (zero) {
      z.push_back(j);
    } else if (l == 0 && use_mf(p)) {
      mf.push_back(p);
      j.C = p->Cbuf;
      j.D = mfDinv<T>(L);
      gather.push_back(j);
    } else if (L.g.N <= p->small_nodes) {
      j.A = opA<T>(L);
      small.push_back(j);
    } else {
      j.A = opA<T>(L);
      j.C = p->Cbuf;
      split.push_back(j);
      lower.push_back(j);
    }
  }
  plan_mf_elements<T>(pl, mf);
  set_mf_gathers(gather, mf);
  pl.add(BOP_PBJ_ZERO, std::move(z));
  pl.add(BOP_DEFECT_SPLIT, std::move(split));
  pl.add(BOP_ROW_SMALL_PBJ, std::move(small));
  pl.add(BOP_MF_GATHER_PBJ, std::move(gather));
  pl.add(BOP_PBJ_LOWER, std::move(lower));
  for (mvpf_problem* p : ps) std::swap(p->lev[l].x, p->lev[l].x2);
}

// r = b - A x on level l of every problem in ps
template <typename T>
void plan_defect(Planner& pl, const std::vector<mvpf_problem*>& ps, int l) {
  std::vector<mvpf_problem*> mf;
  std::vector<BJob> split, lower, small, gather;
  for (mvpf_problem* p : ps) {
    Level& L = p->lev[l];
    BJob j = job_of(L);
    j.D = opD<T>(L);
    j.x = L.x;
    j.b = L.b;
    j.y = L.r;
    if (l == 0 && use_mf(p)) {
      mf.push_back(p);
      j.C = p->Cbuf;
      gather.push_back(j);
    } else if (L.g.N <= p->small_nodes) {
      j.A = opA<T>(L);
      small.push_back(j);
    } else {
      j.A = opA<T>(L);
      j.C = p->Cbuf;
      split.push_back(j);
      lower.push_back(j);
    }
  }
  plan_mf_elements<T>(pl, mf);
  set_mf_gathers(gather, mf);
  pl.add(BOP_DEFECT_SPLIT, std::move(split));
  pl.add(BOP_ROW_SMALL_DEFECT, std::move(small));
  pl.add(BOP_MF_GATHER_DEFECT, std::move(gather));
  pl.add(BOP_DEFECT_LOWER, std::move(lower));
}

template <typename T>
void plan_vcycle(Planner& pl, const std::vector<mvpf_problem*>& ps, int l) {
  std::vector<mvpf_problem*> fine;
  std::vector<BJob> coarse;
  for (mvpf_problem* p : ps) {
    Level& L = p->lev[l];
    if (l == p->L - 1) {
      BJob j = job_of(L);
      j.A = L.Ainv;
      j.b = L.b;
      j.y = L.x;
      coarse.push_back(j);
    } else {
      fine.push_back(p);
    }
  }
  pl.add(BOP_COARSE, std::move(coarse));
  if (fine.empty()) return;
  int nu_pre = 0, nu_post = 0;
  for (mvpf_problem* p : fine) {
    nu_pre = std::max(nu_pre, p->opts.nu_pre);
    nu_post = std::max(nu_post, p->opts.nu_post);
  }
  // pre-smoothing: sweep k of the problems that take more than k sweeps
  std::vector<mvpf_problem*> act;
  for (mvpf_problem* p : fine) {
    if (p->opts.nu_pre > 0) {
      act.push_back(p);
    } else {
      Level& L = p->lev[l];
      T* x = (T*)L.x;
      const int64_t n = nvec(L.g);
      pl.solo([x, n](hipStream_t s) { launch_zero<T>(n, x, s); });
    }
  }
  plan_sweep<T>(pl, act, l, true);
  for (int k = 1; k < nu_pre; ++k) {
    act.clear();
    for (mvpf_problem* p : fine)
      if (p->opts.nu_pre > k) act.push_back(p);
    plan_sweep<T>(pl, act, l, false);
  }
  plan_defect<T>(pl, fine, l);
  std::vector<BJob> rs;
  for (mvpf_problem* p : fine) {
    Level &L = p->lev[l], &C = p->lev[l + 1];
    BJob j{};
    j.g = L.g;
    j.g2 = C.g;
    j.x = L.r;
    j.mask = C.mask;
    j.y = C.b;
    rs.push_back(j);
  }
  pl.add(BOP_RESTRICT, std::move(rs));
  plan_vcycle<T>(pl, fine, l + 1);
  std::vector<BJob> pr;
  for (mvpf_problem* p : fine) {
    Level &L = p->lev[l], &C = p->lev[l + 1];
    BJob j{};
    j.g = L.g;
    j.g2 = C.g;
    j.x = C.x;
    j.mask = L.mask;
    j.y = L.x;
    pr.push_back(j);
  }
  pl.add(BOP_PROLONG, std::move(pr));
  for (int k = 0; k < nu_post; ++k) {
    act.clear();
    for (mvpf_problem* p : fine)
      if (p->opts.nu_post > k) act.push_back(p);
    plan_sweep<T>(pl, act, l, false);
  }
}

// z_i = M_i^-1 v_i for every problem of the batch (v = vin, z = zout)
template <typename T>
void plan_precondition(Planner& pl, mvpf_batch* b) {
  std::vector<BJob> cv, fin;
  for (int i = 0; i < b->n; ++i) {
    Level& L = b->probs[i]->lev[0];
    BJob j = job_of(L);
    j.b = b->vin[i];
    j.y = L.b;
    cv.push_back(j);
  }
  pl.add(BOP_CONVERT, std::move(cv));
  plan_vcycle<T>(pl, b->probs, 0);
  for (int i = 0; i < b->n; ++i) {
    Level& L = b->probs[i]->lev[0];
    BJob j = job_of(L);
    j.x = L.x;
    j.b = b->vin[i];
    j.y = b->zout[i];
    fin.push_back(j);
  }
  pl.add(BOP_FINISH, std::move(fin));
}

template <typename T, typename TZ>
int batch_capture(mvpf_batch* b) {
  batch_drop_graph(b);
  // plan (the sweeps' buffer swaps are replayed on the host, then undone)
  std::vector<std::pair<void*, void*>> saved;
  for (mvpf_problem* p : b->probs)
    for (int l = 0; l < p->L; ++l) saved.emplace_back(p->lev[l].x, p->lev[l].x2);
  Planner pl;
  plan_precondition<T>(pl, b);
  {
    size_t k = 0;
    for (mvpf_problem* p : b->probs)
      for (int l = 0; l < p->L; ++l, ++k) {
        p->lev[l].x = saved[k].first;
        p->lev[l].x2 = saved[k].second;
      }
  }
  // job tables: block ranges, then one upload
  std::vector<BJob> all;
  for (PlanOp& o : pl.ops) {
    if (o.op < 0) continue;
    o.off = all.size();
    int blocks = 0;
    for (BJob& j : o.jobs) {
      j.nblk = batch_job_blocks(o.op, j, o.threads);
      j.block0 = blocks;
      blocks += j.nblk;
      all.push_back(j);
    }
    o.blocks = blocks;
  }
  if (all.size() > b->jobs_cap) {
    if (b->jobs_dev) (void)hipFree(b->jobs_dev);
    b->jobs_dev = nullptr;
    b->jobs_cap = 0;
    if (hipMalloc((void**)&b->jobs_dev, sizeof(BJob) * all.size()) != hipSuccess) {
      (void)hipGetLastError();
      b->err = "batch job table allocation failed";
      return MVPF_ENOMEM;
    }
    b->jobs_cap = all.size();
  }
  if (!all.empty())
    BCHK(hipMemcpy(b->jobs_dev, all.data(), sizeof(BJob) * all.size(), hipMemcpyHostToDevice));
  for (PlanOp& o : pl.ops) {
    if (o.op == BOP_CONVERT) {
      b->conv_off = o.off;
      b->conv_jobs = o.jobs;
    } else if (o.op == BOP_FINISH) {
      b->fin_off = o.off;
      b->fin_jobs = o.jobs;
    }
  }
  hipStream_t s = b->work;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    b->err = "hipStreamBeginCapture failed";
    return MVPF_EDEVICE;
  }
  for (PlanOp& o : pl.ops) {
    if (o.op < 0)
      o.solo(s);
    else
      launch_batch<T, TZ>(o.op, b->jobs_dev + o.off, (int)o.jobs.size(), o.blocks, s, o.threads);
  }
  const bool ok = hipGetLastError() == hipSuccess;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (!ok || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    b->err = "V-cycle graph capture failed";
    return MVPF_EDEVICE;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    batch_drop_graph(b);
    b->err = "V-cycle graph instantiation failed";
    return MVPF_EDEVICE;
  }
  for (int i = 0; i < b->n; ++i) b->graph_version[i] = b->probs[i]->config_version;
  return 0;
}

// Lockstep FGMRES over the batch, all on the batch's work stream.  Per
// Arnoldi step: one launch normalises every problem's new basis vector, one
// graph launch runs all V-cycles (its input and output job entries rewritten
// to point at each problem's v_j and z_j), and every further operation of
// the step -- operator product, both Gram-Schmidt passes, norms, the copy of
// the Hessenberg columns -- is one launch for all problems, followed by one
// device-to-host copy and one synchronisation.  Per-problem work is left
// only where problems are out of step (cycle ends, true residual checks).
constexpr int KOPS_PER_STEP = 9;
constexpr int HCOL = 3 * (MAX_RESTART + 2);

int batch_step_buffers(mvpf_batch* b) {
  if (b->kjobs_dev) return 0;
  const int n = b->n;
  const size_t kb = sizeof(KJob) * KOPS_PER_STEP * n, ob = sizeof(BJob) * 2 * n;
  if (hipMalloc((void**)&b->kjobs_dev, kb) != hipSuccess || hipMalloc((void**)&b->ojobs_dev, ob) != hipSuccess ||
      hipMalloc((void**)&b->bcol_dev, sizeof(double) * HCOL * n) != hipSuccess ||
      hipHostMalloc((void**)&b->kjobs_host, kb) != hipSuccess ||
      hipHostMalloc((void**)&b->ojobs_host, ob) != hipSuccess ||
      hipHostMalloc((void**)&b->gjobs_host, sizeof(BJob) * 2 * n) != hipSuccess ||
      hipHostMalloc((void**)&b->bcol_host, sizeof(double) * HCOL * n) != hipSuccess) {
    (void)hipGetLastError();
    b->err = "batch step buffers allocation failed";
    return MVPF_ENOMEM;
  }
  return 0;
}

// ops of one step over a staged job table: (op, first job, jobs, workgroups)
template <typename J>
struct StepOps {
  J* host;
  std::vector<int> op, first, count, blocks, threads;
  int used = 0;
  template <typename BlocksFn>
  void add(int o, const std::vector<J>& jobs, BlocksFn nblk, int nthreads = 256) {
    if (jobs.empty()) return;
    op.push_back(o);
    first.push_back(used);
    count.push_back((int)jobs.size());
    threads.push_back(nthreads);
    int bl = 0;
    for (J j : jobs) {
      j.nblk = nblk(o, j, nthreads);
      j.block0 = bl;
      bl += j.nblk;
      host[used++] = j;
    }
    blocks.push_back(bl);
  }
};

template <typename T, typename TZ>
int batch_fgmres(mvpf_batch* b, mvpf_solve_stats* st) {
  bool stale = !b->exec;
  for (int i = 0; i < b->n && !stale; ++i) stale = b->graph_version[i] != b->probs[i]->config_version;
  if (stale) TRY((batch_capture<T, TZ>(b)));
  TRY(batch_step_buffers(b));
  hipStream_t s = b->work;
  const int nprob = b->n;
  std::vector<Krylov<T, TZ>> K(nprob);
  for (int i = 0; i < nprob; ++i) {
    mvpf_problem* p = b->probs[i];
    K[i].defer = true;
    TRY(K[i].begin(p, p->rhs, p->dx, &st[i]));
  }
  BCHK(hipStreamSynchronize(s));
  for (auto& k : K) k.after_begin();
  using KP = typename Krylov<T, TZ>::Phase;
  auto kblocks = [](int o, const KJob& j, int) { return krylov_job_blocks(o, j); };
  auto bblocks = [](int o, const BJob& j, int threads) { return batch_job_blocks(o, j, threads); };
  while (true) {
    bool any = false, arnoldi = false;
    for (auto& k : K) {
      any = any || k.phase != KP::DONE;
      arnoldi = arnoldi || k.phase == KP::ARNOLDI;
    }
    if (!any) break;
    if (arnoldi) {
      StepOps<KJob> pre{b->kjobs_host}, post{b->kjobs_host};
      StepOps<BJob> outer{b->ojobs_host};
      // normalisations left by the last step
      std::vector<KJob> sc;
      for (auto& k : K)
        if (k.pend_w) {
          KJob j{};
          j.n = k.n;
          j.w = k.pend_w;
          j.a = k.pend_a;
          sc.push_back(j);
          k.pend_w = nullptr;
        }
      pre.add(KOP_SCALE, sc, kblocks);
      // the V-cycles' ends
      for (int i = 0; i < nprob; ++i) {
        const bool a = K[i].phase == KP::ARNOLDI;
        BJob c = b->conv_jobs[i], f = b->fin_jobs[i];
        c.b = a ? (const void*)K[i].vj() : (const void*)b->vin[i];
        f.b = c.b;  // v itself on constrained dofs
        f.y = a ? (void*)K[i].zj() : b->zout[i];
        b->gjobs_host[i] = c;
        b->gjobs_host[nprob + i] = f;
      }
      // operator product w = A z_j
      std::vector<BJob> oe, og;
      std::vector<mvpf_problem*> omf;
      std::vector<std::function<void(hipStream_t)>> solos;
      for (int i = 0; i < nprob; ++i) {
        if (K[i].phase != KP::ARNOLDI) continue;
        mvpf_problem* p = b->probs[i];
        Level& L0 = p->lev[0];
        const TZ* z = K[i].zj();
        double* w = p->V + (int64_t)(K[i].j + 1) * K[i].n;
        if (use_mf(p)) {
          BJob j{};
          j.g = L0.g;
          j.A = p->Dmf64;
          j.x = z;
          j.mask = L0.mask;
          j.cd = p->card;
          j.C = p->Cbuf;
          j.y = w;
          oe.push_back(j);
          og.push_back(j);
          omf.push_back(p);
          if (contact(p))
            solos.push_back([p, z](hipStream_t st_) {
              Level& L = p->lev[0];
              launch_contact_apply<double, TZ>(L.g, p->sphere, L.state, L.mask, z, (double*)p->Cbuf, st_);
            });
        } else {
          solos.push_back([p, z, w](hipStream_t st_) {
            launch_spmv<double, TZ, double>(p->lev[0].g, p->lev[0].A64, z, w, p->Cbuf, st_, p->outer_G);
          });
        }
      }
      set_mf_gathers(og, omf);
      outer.add(BOP_MF_OUTER_ELEMENT, oe, bblocks, 8 * batch_mf_epw(omf));
      outer.add(BOP_MF_OUTER_GATHER, og, bblocks);
      // classical Gram-Schmidt twice, norm, Hessenberg columns
      std::vector<KJob> md, rd1, ax1, rd2, ax2, rdn, cp;
      for (int i = 0; i < nprob; ++i) {
        auto& k = K[i];
        if (k.phase != KP::ARNOLDI) continue;
        mvpf_problem* p = b->probs[i];
        KJob j{};
        j.n = k.n;
        j.V = p->V;
        j.w = p->V + (int64_t)(k.j + 1) * k.n;
        j.part = p->red;
        j.k = k.j + 1;
        j.nb = k.nb;
        md.push_back(j);
        KJob r = j;
        r.out = k.h1();
        rd1.push_back(r);
        KJob a = j;
        a.h = k.h1();
        ax1.push_back(a);
        r.out = k.h2();
        rd2.push_back(r);
        a.h = k.h2();
        a.flag = 1;
        ax2.push_back(a);
        r.out = k.hn();
        r.k = 1;
        rdn.push_back(r);
        KJob c{};
        c.src = p->hcol;
        c.out = b->bcol_dev + (int64_t)i * HCOL;
        c.k = HCOL;
        cp.push_back(c);
      }
      post.used = pre.used;
      post.add(KOP_MULTIDOT, md, kblocks);
      post.add(KOP_REDUCE, rd1, kblocks);
      post.add(KOP_MULTIAXPY, ax1, kblocks);
      post.add(KOP_MULTIDOT, md, kblocks);
      post.add(KOP_REDUCE, rd2, kblocks);
      post.add(KOP_MULTIAXPY, ax2, kblocks);
      post.add(KOP_REDUCE, rdn, kblocks);
      post.add(KOP_COPY, cp, kblocks);
      // stage, then launch in order
      BCHK(hipMemcpyAsync(b->kjobs_dev, b->kjobs_host, sizeof(KJob) * post.used, hipMemcpyHostToDevice, s));
      if (outer.used)
        BCHK(hipMemcpyAsync(b->ojobs_dev, b->ojobs_host, sizeof(BJob) * outer.used, hipMemcpyHostToDevice, s));
      BCHK(hipMemcpyAsync(b->jobs_dev + b->conv_off, b->gjobs_host, sizeof(BJob) * nprob, hipMemcpyHostToDevice, s));
      BCHK(hipMemcpyAsync(b->jobs_dev + b->fin_off, b->gjobs_host + nprob, sizeof(BJob) * nprob,
                          hipMemcpyHostToDevice, s));
      for (size_t q = 0; q < pre.op.size(); ++q)
        launch_krylov_batch(pre.op[q], b->kjobs_dev + pre.first[q], pre.count[q], pre.blocks[q], s);
      BCHK(hipGraphLaunch(b->exec, s));
      // element launches, then the per-problem contact and product launches, then the gather
      size_t q = 0;
      for (; q < outer.op.size() && outer.op[q] == BOP_MF_OUTER_ELEMENT; ++q)
        launch_batch<T, TZ>(outer.op[q], b->ojobs_dev + outer.first[q], outer.count[q], outer.blocks[q], s,
                            outer.threads[q]);
      for (auto& f : solos) f(s);
      for (; q < outer.op.size(); ++q)
        launch_batch<T, TZ>(outer.op[q], b->ojobs_dev + outer.first[q], outer.count[q], outer.blocks[q], s,
                            outer.threads[q]);
      for (size_t q = 0; q < post.op.size(); ++q)
        launch_krylov_batch(post.op[q], b->kjobs_dev + post.first[q], post.count[q], post.blocks[q], s);
      BCHK(hipGetLastError());
      BCHK(hipMemcpyAsync(b->bcol_host, b->bcol_dev, sizeof(double) * HCOL * nprob, hipMemcpyDeviceToHost, s));
    }
    BCHK(hipStreamSynchronize(s));
    for (int i = 0; i < nprob; ++i) {
      auto& k = K[i];
      if (k.phase == KP::ARNOLDI) {
        std::memcpy(k.p->hhost, b->bcol_host + (int64_t)i * HCOL, sizeof(double) * HCOL);
        TRY(k.arnoldi_finish());
      } else if (k.phase == KP::CHECK) {
        k.check_finish();
      }
    }
  }
  int rc = 0;
  for (auto& k : K)
    if (k.rc) rc = k.rc;
  return rc;
}

// ---- batched Newton systems ----------------------------------------------------
// The heavy assembly kernels (Gauss-point Hessians, element matrices, block
// gathers, symmetric elimination, Hessian pack, residual rows, block
// inverses) run as one launch per kernel and level for all problems, level
// by level from each problem's coarsest; the light per-problem steps (masks,
// injections, dense coarse gather, contact terms, lifting, right-hand side)
// stay per problem.  Same kernels and arithmetic per problem as
// build_system, so the systems are bitwise the same.  All on one stream; the
// batched coarse inversion overlaps on the work stream once every coarsest
// level is assembled.  Needs every level of every problem in one slab.
bool batch_single_slabs(const mvpf_batch* b) {
  for (const mvpf_problem* p : b->probs)
    for (int l = 0; l < p->L; ++l)
      if (make_chunks(p->lev[l].g, p->ne_use).size() != 1) return false;
  return true;
}

struct AsmStep {
  int op = -1;  // AssemblyOp, or -1 for host code that enqueues per-problem work
  int pade = 22;
  size_t first = 0;
  int count = 0, blocks = 0;
  std::function<int()> host;
};

int batch_assemble(mvpf_batch* b, const double* depths, hipStream_t s) {
  std::vector<AsmStep> steps;
  std::vector<AJob> all;
  auto add = [&](int op, int pade, const std::vector<AJob>& jobs, const std::vector<char>& diag) {
    if (jobs.empty()) return;
    AsmStep st;
    st.op = op;
    st.pade = pade;
    st.first = all.size();
    st.count = (int)jobs.size();
    for (size_t k = 0; k < jobs.size(); ++k) {
      AJob j = jobs[k];
      j.nblk = assembly_job_blocks(op, j, !diag.empty() && diag[k]);
      j.block0 = st.blocks;
      st.blocks += j.nblk;
      all.push_back(j);
    }
    steps.push_back(st);
  };
  auto host = [&](std::function<int()> f) {
    AsmStep st;
    st.host = std::move(f);
    steps.push_back(std::move(st));
  };
  auto job = [](mvpf_problem* p, int l) {
    Level& L = p->lev[l];
    AJob j{};
    j.g = L.g;
    j.ck = make_chunks(L.g, p->ne_use)[0];
    j.state = L.state;
    j.cd = p->card;
    j.qp = p->qp;
    j.elem = p->elem;
    j.A64 = L.A64;
    j.A32 = L.A32;
    j.diag64 = L.diag64;
    j.mask = L.mask;
    return j;
  };
  auto qp_steps = [&](const std::vector<mvpf_problem*>& ps, const std::vector<AJob>& js) {
    for (int mix : {0, 1})
      for (int pd : {11, 22, 33}) {
        std::vector<AJob> sel;
        for (size_t k = 0; k < ps.size(); ++k)
          if ((ps[k]->pade == pd || (pd == 22 && ps[k]->pade != 11 && ps[k]->pade != 33)) && ps[k]->mixing == mix)
            sel.push_back(js[k]);
        add(AOP_QP_HESS, pd + mix * QP_LOG_MIX, sel, {});
      }
  };
  const int n = b->n;
  int maxL = 0;
  for (mvpf_problem* p : b->probs) maxL = std::max(maxL, p->L);
  for (int i = 0; i < n; ++i) {
    mvpf_problem* p = b->probs[i];
    const double d = depths[i];
    host([p, d] { return system_prelude(p, d); });
  }
  // coarse levels, each problem's coarsest first
  for (int k = 0; k < maxL - 1; ++k) {
    std::vector<mvpf_problem*> ps;
    std::vector<AJob> js;
    std::vector<int> lv;
    for (mvpf_problem* p : b->probs) {
      const int l = p->L - 1 - k;
      if (l < 1) continue;
      ps.push_back(p);
      js.push_back(job(p, l));
      lv.push_back(l);
    }
    qp_steps(ps, js);
    add(AOP_ELEMENT, 0, js, {});
    for (size_t q = 0; q < ps.size(); ++q)
      if (contact(ps[q])) {
        mvpf_problem* p = ps[q];
        const int l = lv[q];
        const double d = depths[std::find(b->probs.begin(), b->probs.end(), p) - b->probs.begin()];
        host([p, l, d] {
          Level& C = p->lev[l];
          launch_contact_element(C.g, make_chunks(C.g, p->ne_use)[0], make_sphere(C.g, p->load, d), C.state,
                                 p->elem, p->stream);
          return 0;
        });
      }
    add(AOP_GATHER, 0, js, {});
    add(AOP_DIRICHLET, 0, js, {});
    if (k == 0) {
      // every coarsest operator into its dense matrix (inverted below)
      host([b, s]() -> int {
        for (mvpf_problem* p : b->probs) {
          Level& C = p->lev[p->L - 1];
          launch_dense_from_bsr(C.g, C.A64, p->coarse_work ? p->coarse_work : p->V, s);
          p->coarse_pending = false;
        }
        BCHK(hipEventRecord(b->fork, s));
        return 0;
      });
    }
  }
  // finest level: only the diagonal blocks on matrix-free levels
  {
    std::vector<AJob> js, pk;
    std::vector<char> diag;
    for (mvpf_problem* p : b->probs) {
      AJob j = job(p, 0);
      j.R = p->R;
      js.push_back(j);
      diag.push_back(use_mf(p) ? 1 : 0);
      if (use_mf(p)) {
        AJob q = j;
        q.D64 = p->Dmf64;
        q.D32 = p->Dmf32;
        pk.push_back(q);
      }
    }
    qp_steps(b->probs, js);
    add(AOP_MF_PACK, 0, pk, {});
    add(AOP_RESIDUAL, 0, js, {});
    add(AOP_ELEMENT, 0, js, diag);
    for (int i = 0; i < n; ++i)
      if (contact(b->probs[i])) {
        mvpf_problem* p = b->probs[i];
        const double d = depths[i];
        host([p, d] {
          Level& L0 = p->lev[0];
          launch_contact_element(L0.g, make_chunks(L0.g, p->ne_use)[0], make_sphere(L0.g, p->load, d), L0.state,
                                 p->elem, p->stream, use_mf(p));
          return 0;
        });
      }
    std::vector<AJob> ga = js;
    for (size_t q = 0; q < ga.size(); ++q)
      if (diag[q]) ga[q].A64 = nullptr, ga[q].A32 = nullptr;  // diagonal blocks only
    add(AOP_GATHER, 0, ga, diag);
    for (int i = 0; i < n; ++i) {
      mvpf_problem* p = b->probs[i];
      const double d = depths[i];
      host([p, d] { return system_rhs(p, d); });
    }
    add(AOP_DIRICHLET, 0, js, {});
  }
  // smoother setup on every level but the coarsest, the inversions, the join
  {
    std::vector<AJob> bi;
    for (mvpf_problem* p : b->probs)
      for (int l = 0; l < p->L - 1; ++l) {
        Level& L = p->lev[l];
        AJob j{};
        j.g = L.g;
        j.diag64 = L.diag64;
        j.Dinv64 = L.Dinv64;
        j.Dinv32 = L.Dinv32;
        j.DinvS32 = L.DinvS32;
        j.status = setup_status(p);
        bi.push_back(j);
      }
    add(AOP_BLOCK_INVERSE, 0, bi, {});
    // all coarsest-level inversions at once on the work stream, enqueued
    // after the assembly so that the host feeds the assembly stream first
    host([b]() -> int {
      BCHK(hipStreamWaitEvent(b->work, b->fork, 0));
      if (dense_invert_batch(b->gj_tab, b->gj_sel, b->gj_n, b->work) != 0) {
        b->err = "batched coarse inversion launch failed";
        return MVPF_EDEVICE;
      }
      BCHK(hipEventRecord(b->leave, b->work));
      return 0;
    });
    host([b, s]() -> int {
      BCHK(hipStreamWaitEvent(s, b->leave, 0));
      for (mvpf_problem* p : b->probs)
        HIPCHK(hipMemcpyAsync(host_status(p), setup_status(p), sizeof(int), hipMemcpyDeviceToHost, s));
      return 0;
    });
  }
  // one upload of all job tables, then the steps in order
  if (all.size() > b->ajobs_cap) {
    if (b->ajobs_dev) (void)hipFree(b->ajobs_dev);
    b->ajobs_dev = nullptr;
    b->ajobs_cap = 0;
    if (hipMalloc((void**)&b->ajobs_dev, sizeof(AJob) * all.size()) != hipSuccess) {
      (void)hipGetLastError();
      b->err = "batch assembly job table allocation failed";
      return MVPF_ENOMEM;
    }
    b->ajobs_cap = all.size();
  }
  BCHK(hipMemcpy(b->ajobs_dev, all.data(), sizeof(AJob) * all.size(), hipMemcpyHostToDevice));
  for (AsmStep& st : steps) {
    if (st.op < 0) {
      const int rc = st.host();
      if (rc) {
        if (b->err.empty()) b->err = "batched assembly failed";
        return rc;
      }
    } else {
      launch_assembly_batch(st.op, st.pade, b->ajobs_dev + st.first, st.count, st.blocks, s);
    }
  }
  BCHK(hipGetLastError());
  return 0;
}

void batch_free(mvpf_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  for (double*& v : b->vin) dfree(v);
  for (void*& z : b->zout) {
    if (z) (void)hipFree(z);
    z = nullptr;
  }
  for (hipStream_t& st : b->branch)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t& e : b->join)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->enter) (void)hipEventDestroy(b->enter);
  if (b->leave) (void)hipEventDestroy(b->leave);
  if (b->gj_tab) (void)hipFree(b->gj_tab);
  if (b->gj_sel) (void)hipFree(b->gj_sel);
  if (b->jobs_dev) (void)hipFree(b->jobs_dev);
  b->jobs_dev = nullptr;
  b->jobs_cap = 0;
  for (void* d : {(void*)b->kjobs_dev, (void*)b->ojobs_dev, (void*)b->bcol_dev, (void*)b->ajobs_dev})
    if (d) (void)hipFree(d);
  b->ajobs_dev = nullptr;
  b->ajobs_cap = 0;
  for (void* h : {(void*)b->kjobs_host, (void*)b->ojobs_host, (void*)b->gjobs_host, (void*)b->bcol_host})
    if (h) (void)hipHostFree(h);
  b->kjobs_dev = nullptr;
  b->ojobs_dev = nullptr;
  b->bcol_dev = nullptr;
  b->kjobs_host = nullptr;
  b->ojobs_host = nullptr;
  b->gjobs_host = nullptr;
  b->bcol_host = nullptr;
  b->gj_tab = nullptr;
  b->gj_sel = nullptr;
  if (b->work) {
    (void)hipStreamSynchronize(b->work);
    (void)hipStreamDestroy(b->work);
  }
  b->work = nullptr;
  for (mvpf_problem* p : b->probs)
    if (p) mvpf_destroy(p);
  b->probs.clear();
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

void mvpf_default_opts(mvpf_opts* o) {
  if (!o) return;
  o->precision = MVPF_FP64;
  o->rtol = 1e-8;
  o->restart = 30;
  o->max_it = 500;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->omega = 0.55;
  o->newton_max = 12;
  o->newton_rtol = 1e-9;
  o->coarse = MVPF_COARSE_REDISCRETISE;
}

int mvpf_nvar(void) { return NV; }

int mvpf_create(const mvpf_mesh* mesh, const mvpf_material* mat, const mvpf_loading* load, const mvpf_opts* opts,
                void* stream, mvpf_problem** out) {
  if (!out) return MVPF_EINVAL;
  *out = nullptr;
  std::string err;
  int rc = validate(mesh, mat, load, opts, err);
  if (!rc && NV != 6) {
    err = "the six-variant material card needs a library built for six variants (this one has " +
          std::to_string(NV) + "); use mvpf_create_orbit";
    rc = MVPF_EINVAL;
  }
  if (rc) {
    g_create_err = err;
    return rc;
  }
  mvpf_problem* p = new mvpf_problem();
  p->mesh = *mesh;
  p->mat = *mat;
  p->load = *load;
  p->opts = *opts;
  p->stream = (hipStream_t)stream;
  rc = allocate(p);
  if (rc) {
    g_create_err = p->err;
    destroy_all(p);
    delete p;
    return rc;
  }
  *out = p;
  return 0;
}

int mvpf_create_orbit(const mvpf_mesh* mesh, const mvpf_orbit_material* om, const mvpf_loading* load,
                      const mvpf_opts* opts, void* stream, mvpf_problem** out) {
  if (!out) return MVPF_EINVAL;
  *out = nullptr;
  if (!om) {
    g_create_err = "null argument";
    return MVPF_EINVAL;
  }
  // the checks that do not depend on the kind of card
  mvpf_material shape{};
  shape.pade = om->pade;
  shape.mixing = om->mixing;
  std::string err;
  int rc = validate(mesh, &shape, load, opts, err);
  if (!rc) {
    DevCard probe;
    const int n = build_card_orbit(*om, probe);
    if (n != NV) {
      err = "the cubic orbit of U1 has " + std::to_string(n) + " variants; this library is built for " +
            std::to_string(NV);
      rc = MVPF_EINVAL;
    }
  }
  if (rc) {
    g_create_err = err;
    return rc;
  }
  mvpf_problem* p = new mvpf_problem();
  p->mesh = *mesh;
  p->mat = shape;
  p->mat.rho = om->rho;
  p->omat = *om;
  p->orbit = true;
  p->load = *load;
  p->opts = *opts;
  p->stream = (hipStream_t)stream;
  rc = allocate(p);
  if (rc) {
    g_create_err = p->err;
    destroy_all(p);
    delete p;
    return rc;
  }
  *out = p;
  return 0;
}

void mvpf_destroy(mvpf_problem* p) {
  if (!p) return;
  destroy_all(p);
  delete p;
}

const char* mvpf_last_error(const mvpf_problem* p) { return p ? p->err.c_str() : g_create_err.c_str(); }

int mvpf_get_info(const mvpf_problem* p, mvpf_info* info) {
  if (!p || !info) return MVPF_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->n_levels = p->L;
  for (int l = 0; l < p->L; ++l) {
    info->nx[l] = p->lev[l].g.nx;
    info->ny[l] = p->lev[l].g.ny;
    info->nz[l] = p->lev[l].g.nz;
    info->n_nodes[l] = p->lev[l].g.N;
  }
  info->bytes_device = p->bytes;
  return 0;
}

int mvpf_set_opts(mvpf_problem* p, const mvpf_opts* o) {
  if (!p || !o) return MVPF_EINVAL;
  std::string err;
  int rc = validate(&p->mesh, &p->mat, &p->load, o, err);
  if (rc) { p->err = err; return rc; }
  if (o->precision != p->opts.precision || o->restart > p->restart_cap) {
    p->err = "precision and a larger restart need a new problem";
    return MVPF_EINVAL;
  }
  p->opts = *o;
  p->config_version++;
  return 0;
}

int mvpf_set_state(mvpf_problem* p, const double* u, const double* eta, const double* eta_prev, double depth) {
  if (!p) return MVPF_EINVAL;
  const Grid& g = p->lev[0].g;
  if (u) launch_interleaved_to_soa(g, u, 3, 0, 3, p->lev[0].state, p->stream);
  if (eta) launch_interleaved_to_soa(g, eta, NV, 3, NV, p->lev[0].state, p->stream);
  if (eta_prev) launch_interleaved_to_soa(g, eta_prev, NV, 3 + NV, NV, p->lev[0].state, p->stream);
  p->depth = depth;
  p->have_system = p->have_solution = false;
  TRY(launch_check(p, "set_state"));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int mvpf_get_state(mvpf_problem* p, double* u, double* eta, double* eta_prev, double* depth) {
  if (!p) return MVPF_EINVAL;
  const Grid& g = p->lev[0].g;
  if (u) launch_soa_to_interleaved(g, p->lev[0].state, 3, 0, 3, u, p->stream);
  if (eta) launch_soa_to_interleaved(g, p->lev[0].state, NV, 3, NV, eta, p->stream);
  if (eta_prev) launch_soa_to_interleaved(g, p->lev[0].state, NV, 3 + NV, NV, eta_prev, p->stream);
  if (depth) *depth = p->depth;
  TRY(launch_check(p, "get_state"));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int mvpf_init_random(mvpf_problem* p, uint64_t seed) {
  if (!p) return MVPF_EINVAL;
  launch_init_random(p->lev[0].g, seed, p->lev[0].state, p->stream);
  p->depth = 0.0;
  p->have_system = p->have_solution = false;
  TRY(launch_check(p, "init_random"));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int mvpf_residual(mvpf_problem* p, double* R, double* norm_free) {
  if (!p) return MVPF_EINVAL;
  TRY(compute_residual(p, p->have_system ? p->sys_depth : p->depth, norm_free));
  if (R) launch_soa_to_interleaved(p->lev[0].g, p->R, NDOF, 0, NDOF, R, p->stream);
  TRY(launch_check(p, "residual"));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int mvpf_newton_system(mvpf_problem* p, double depth) {
  if (!p) return MVPF_EINVAL;
  p->have_system = p->have_solution = false;
  TRY(build_system(p, depth));
  TRY(setup_solver(p));
  p->sys_depth = depth;
  p->have_system = true;
  return 0;
}

int mvpf_get_rhs(mvpf_problem* p, double* b) {
  if (!p || !b) return MVPF_EINVAL;
  if (!p->have_system) { p->err = "no Newton system"; return MVPF_ESTATE; }
  launch_soa_to_interleaved(p->lev[0].g, p->rhs, NDOF, 0, NDOF, b, p->stream);
  TRY(launch_check(p, "get_rhs"));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int mvpf_jacobian_apply(mvpf_problem* p, int level, int precision, const double* x, double* y) {
  if (!p || !x || !y || level < 0 || level >= p->L) return MVPF_EINVAL;
  if (!p->have_system) { p->err = "no Newton system"; return MVPF_ESTATE; }
  Level& L = p->lev[level];
  const Grid& g = L.g;
  hipStream_t s = p->stream;
  launch_interleaved_to_soa(g, x, NDOF, 0, NDOF, p->tmp, s);
  const bool mf = level == 0 && use_mf(p);
  if (precision == MVPF_FP64) {
    if (mf) {
      mf_elements<double, double>(p, p->tmp, true);
      launch_mf_gather<0, double, double, double>(g, (const double*)p->Cbuf, contact(p), p->mf_epw, L.mask, p->tmp,
                                                  nullptr, nullptr, 0.0, p->tmp2, s);
    } else {
      if (!L.A64) { p->err = "no FP64 operator on this level"; return MVPF_EINVAL; }
      launch_spmv<double, double, double>(g, L.A64, p->tmp, p->tmp2, p->Cbuf, s);
    }
  } else if (precision == MVPF_MIXED) {
    if (mf ? !p->Dmf32 : !L.A32) { p->err = "no FP32 operator on this level"; return MVPF_EINVAL; }
    launch_convert<double, float>(nvec(g), p->tmp, (float*)L.x, s);
    if (mf) {
      mf_elements<float, float>(p, (const float*)L.x, true);
      launch_mf_gather<0, float, float, float>(g, (const float*)p->Cbuf, contact(p), p->mf_epw, L.mask,
                                               (const float*)L.x, nullptr, nullptr, 0.0f, (float*)L.r, s);
    } else {
      launch_spmv<float, float, float>(g, L.A32, (const float*)L.x, (float*)L.r, p->Cbuf, s);
    }
    launch_convert<float, double>(nvec(g), (const float*)L.r, p->tmp2, s);
  } else {
    return MVPF_EINVAL;
  }
  launch_soa_to_interleaved(g, p->tmp2, NDOF, 0, NDOF, y, s);
  TRY(launch_check(p, "jacobian_apply"));
  HIPCHK(hipStreamSynchronize(s));
  return 0;
}

int mvpf_precondition(mvpf_problem* p, const double* v, double* z) {
  if (!p || !v || !z) return MVPF_EINVAL;
  if (!p->have_system) { p->err = "no Newton system"; return MVPF_ESTATE; }
  const Grid& g = p->lev[0].g;
  launch_interleaved_to_soa(g, v, NDOF, 0, NDOF, p->tmp, p->stream);
  if (p->mixed)
    precondition<float, double>(p, p->tmp, p->tmp2);
  else
    precondition<double, double>(p, p->tmp, p->tmp2);
  launch_soa_to_interleaved(g, p->tmp2, NDOF, 0, NDOF, z, p->stream);
  TRY(launch_check(p, "precondition"));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

int mvpf_solve(mvpf_problem* p, const double* b, double* x, mvpf_solve_stats* stats) {
  if (!p) return MVPF_EINVAL;
  if (!p->have_system) { p->err = "no Newton system"; return MVPF_ESTATE; }
  mvpf_solve_stats local;
  mvpf_solve_stats* st = stats ? stats : &local;
  const Grid& g = p->lev[0].g;
  const double* bb = p->rhs;
  if (b) {
    launch_interleaved_to_soa(g, b, NDOF, 0, NDOF, p->tmp2, p->stream);
    bb = p->tmp2;
  }
  int rc = solve_internal(p, bb, p->dx, st);
  if (rc < 0) return rc;
  if (x) {
    launch_soa_to_interleaved(g, p->dx, NDOF, 0, NDOF, x, p->stream);
    TRY(launch_check(p, "solve output"));
    HIPCHK(hipStreamSynchronize(p->stream));
  }
  p->have_solution = (b == nullptr);
  if (rc == MVPF_ENOTCONV) p->err = "FGMRES reached max_it";
  return rc;
}

int mvpf_newton_update(mvpf_problem* p) {
  if (!p) return MVPF_EINVAL;
  if (!p->have_solution) { p->err = "no Newton increment"; return MVPF_ESTATE; }
  Level& L0 = p->lev[0];
  launch_state_update(L0.g, L0.mask, L0.target, p->dx, L0.state, p->stream);
  TRY(launch_check(p, "newton_update"));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->depth = p->sys_depth;
  p->have_solution = false;
  p->have_system = false;
  return 0;
}

int mvpf_newton_step(mvpf_problem* p, double depth, mvpf_solve_stats* stats) {
  if (!p) return MVPF_EINVAL;
  TRY(mvpf_newton_system(p, depth));
  const int rc = mvpf_solve(p, nullptr, nullptr, stats);
  if (rc < 0) return rc;
  TRY(mvpf_newton_update(p));
  return rc;
}

}  // extern "C"

namespace {

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Newton iterations of one implicit step to indenter depth `trial` from the
// current state (Sec. 3.4): system, solve, update until the free-dof residual
// is <= newton_rtol ||b_0|| (b_0 = the first right-hand side), checked before
// each of at most newton_max solves and after the last (a linear solve that
// stops at max_it still gives the update: an inexact Newton step).  A
// non-finite residual or a singular 9x9 block / coarse operator ends the
// iterations without success (*ok false, return 0); other errors are
// returned.  Timings and iteration counts accumulate into st; *its = the
// solves made.
int newton_iterate(mvpf_problem* p, double trial, mvpf_step_stats* st, int* its, bool* ok, EventPair& ev) {
  Level& L0 = p->lev[0];
  double b0 = 0.0;
  for (int it = 0; it <= p->opts.newton_max; ++it) {
    double rfree = 0.0;
    TRY(compute_residual(p, trial, &rfree));
    st->residual = rfree;
    if (!std::isfinite(rfree)) return 0;
    if (it > 0 && rfree <= p->opts.newton_rtol * b0) {
      *ok = true;
      return 0;
    }
    if (it == p->opts.newton_max) return 0;
    (void)hipEventRecord(ev.a, p->stream);
    TRY(build_system(p, trial));
    (void)hipEventRecord(ev.b, p->stream);
    (void)hipEventSynchronize(ev.b);
    st->assemble_ms += elapsed_ms(ev.a, ev.b);
    (void)hipEventRecord(ev.a, p->stream);
    const int srs = setup_solver(p);
    (void)hipEventRecord(ev.b, p->stream);
    (void)hipEventSynchronize(ev.b);
    st->setup_ms += elapsed_ms(ev.a, ev.b);
    if (srs == MVPF_ESINGULAR) return 0;  // a failed attempt: the caller halves the increment
    TRY(srs);
    p->sys_depth = trial;
    p->have_system = true;
    if (it == 0) {
      TRY(norm_device(p, nvec(L0.g), p->rhs, &b0));
      st->residual0 = b0;
    }
    mvpf_solve_stats ss;
    TRY(solve_internal(p, p->rhs, p->dx, &ss));
    st->linear_iterations += ss.iterations;
    st->solve_ms += ss.solve_ms;
    st->newton_iterations++;
    (*its)++;
    p->have_solution = true;
    TRY(mvpf_newton_update(p));
  }
  return 0;
}

// One implicit step to indenter depth `trial` (newton_iterate).  On success
// eta_hat_n <- eta_hat and the depth becomes `trial`.  On every other exit --
// no convergence, a singular block, or an error returned by any call after
// the state was saved -- the state and the depth are restored to their
// values at entry before returning.
int newton_attempt(mvpf_problem* p, double trial, mvpf_step_stats* st, int* its, bool* ok) {
  Level& L0 = p->lev[0];
  const size_t sbytes = sizeof(double) * NSTATE * L0.g.Npad;
  EventPair ev;
  *ok = false;
  *its = 0;
  const double depth0 = p->depth;  // the updates move it with the state
  HIPCHK(hipMemcpyAsync(p->save_state, L0.state, sbytes, hipMemcpyDeviceToDevice, p->stream));
  const int rc = newton_iterate(p, trial, st, its, ok, ev);
  if (rc == 0 && *ok) {
    HIPCHK(hipMemcpyAsync(L0.state + (int64_t)(3 + NV) * L0.g.Npad, L0.state + (int64_t)3 * L0.g.Npad,
                          sizeof(double) * NV * L0.g.Npad, hipMemcpyDeviceToDevice, p->stream));
    p->depth = trial;
  } else {
    *ok = false;
    if (p->coarse_pending) {  // an error between the coarse inversion's fork and its join
      (void)hipStreamWaitEvent(p->stream, p->ev_join, 0);
      p->coarse_pending = false;
    }
    const hipError_t e = hipMemcpyAsync(L0.state, p->save_state, sbytes, hipMemcpyDeviceToDevice, p->stream);
    p->depth = depth0;
    if (rc == 0 && e != hipSuccess) {
      p->err = std::string("state restore failed: ") + hipGetErrorString(e);
      return MVPF_EDEVICE;
    }
  }
  const hipError_t es = hipStreamSynchronize(p->stream);
  p->have_system = p->have_solution = false;
  if (rc != 0) return rc;
  if (es != hipSuccess) {
    p->err = std::string("hipStreamSynchronize failed: ") + hipGetErrorString(es);
    return MVPF_EDEVICE;
  }
  return 0;
}

// viscous coefficient rho of the material card (time-step dependent)
int set_rho(mvpf_problem* p, double rho) {
  p->mat.rho = rho;
  p->omat.rho = rho;
  DevCard hc;
  make_card(p, hc);
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipMemcpy(p->card, &hc, sizeof(DevCard), hipMemcpyHostToDevice));
  return 0;
}

int contact_load(mvpf_problem* p, double depth, double* P) {
  Level& L0 = p->lev[0];
  launch_contact_load(L0.g, make_sphere(L0.g, p->load, depth), L0.state, p->tmp, p->stream);
  TRY(launch_check(p, "contact load"));
  HIPCHK(hipMemcpyAsync(P, p->tmp, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

}  // namespace

extern "C" {

int mvpf_time_step(mvpf_problem* p, double depth, mvpf_step_stats* stats) {
  if (!p) return MVPF_EINVAL;
  mvpf_step_stats local;
  mvpf_step_stats* st = stats ? stats : &local;
  std::memset(st, 0, sizeof(*st));
  const double goal = depth;
  const double rho0 = p->orbit ? p->omat.rho : p->mat.rho;
  const double dd0 = std::fabs(goal - p->depth);  // the increment the material's rho belongs to
  double trial = depth;
  int rc = 0;
  while (true) {
    const double cur = p->depth;
    // rho = 1/(m tau) and tau is proportional to the increment: a halved
    // increment doubles rho (the last attempt to the goal uses rho0 again)
    const double dd = std::fabs(trial - cur);
    const double rho = (dd > 0 && dd < dd0) ? rho0 * (dd0 / dd) : rho0;
    if ((rc = set_rho(p, rho)) != 0) break;
    bool ok = false;
    int its = 0;
    if ((rc = newton_attempt(p, trial, st, &its, &ok)) != 0) break;
    if (ok) {
      if (trial == goal) {
        st->converged = 1;
        break;
      }
      trial = goal;
      continue;
    }
    if (++st->halvings > 8) {
      p->err = "Newton failed after 8 halvings";
      rc = MVPF_ENOTCONV;
      break;
    }
    trial = cur + 0.5 * (trial - cur);
  }
  if ((p->orbit ? p->omat.rho : p->mat.rho) != rho0) {
    const int rr = set_rho(p, rho0);
    if (rc == 0) rc = rr;
  }
  return rc;
}

int mvpf_set_viscosity(mvpf_problem* p, double rho) {
  if (!p) return MVPF_EINVAL;
  if (!std::isfinite(rho) || rho < 0) {
    p->err = "viscosity: rho must be finite and >= 0";
    return MVPF_EINVAL;
  }
  return set_rho(p, rho);
}

int mvpf_contact_load(mvpf_problem* p, double* load) {
  if (!p || !load) return MVPF_EINVAL;
  if (!contact(p)) {
    p->err = "the indentation load needs the sphere-contact loading";
    return MVPF_EINVAL;
  }
  return contact_load(p, p->depth, load);
}

void mvpf_default_indent_opts(mvpf_indent_opts* o) {
  if (!o) return;
  o->depth_max = 0.05;
  o->unload = 1;
  o->dd_init = 0.0025;
  o->dd_min = 1e-5;
  o->dd_max = 0.01;
  o->grow = 1.25;
  o->shrink = 0.8;
  o->newton_desired = 7;
  o->visc_depth = 2.857e-4;
  o->max_steps = 1000;
}

int mvpf_indent(mvpf_problem* p, const mvpf_indent_opts* o, mvpf_indent_callback on_step, void* user,
                mvpf_indent_record* rec, int max_rec, int* n_rec) {
  if (!p || !o || !n_rec || (max_rec > 0 && !rec)) return MVPF_EINVAL;
  *n_rec = 0;
  if (!contact(p)) {
    p->err = "indentation needs the sphere-contact loading";
    return MVPF_EINVAL;
  }
  if (!(o->depth_max > p->depth) || !(o->dd_min > 0) || !(o->dd_init >= o->dd_min) || !(o->dd_max >= o->dd_init) ||
      !(o->grow >= 1.0) || !(o->shrink > 0.0 && o->shrink <= 1.0) || !(o->visc_depth > 0) || o->max_steps < 1 ||
      max_rec < o->max_steps) {
    p->err = "bad indentation options";
    return MVPF_EINVAL;
  }
  const double rho0 = p->orbit ? p->omat.rho : p->mat.rho;
  double dd = o->dd_init;
  const double goals[2] = {o->depth_max, 0.0};
  int rc = 0, rejected = 0;
  for (int ph = 0; ph < (o->unload ? 2 : 1) && rc == 0; ++ph) {
    const double goal = goals[ph];
    const double sign = goal > p->depth ? 1.0 : -1.0;
    while (p->depth != goal) {
      if (*n_rec >= o->max_steps) {
        p->err = "indentation: step limit reached";
        rc = MVPF_ENOTCONV;
        break;
      }
      const double rem = std::fabs(goal - p->depth);
      double step, trial;
      if (rem <= dd + o->dd_min) {  // the phase's last step lands on its goal
        step = rem;
        trial = goal;
      } else {
        step = dd;
        trial = p->depth + sign * dd;
      }
      if ((rc = set_rho(p, o->visc_depth / step)) != 0) break;
      mvpf_step_stats st;
      std::memset(&st, 0, sizeof(st));
      bool ok = false;
      int its = 0;
      if ((rc = newton_attempt(p, trial, &st, &its, &ok)) != 0) break;
      if (!ok) {
        ++rejected;
        dd = 0.5 * step;
        if (dd < o->dd_min) {
          p->err = "indentation: step below dd_min";
          rc = MVPF_ENOTCONV;
          break;
        }
        continue;
      }
      mvpf_indent_record& r = rec[*n_rec];
      r.depth = p->depth;
      if ((rc = contact_load(p, p->depth, &r.load)) != 0) break;
      r.dd = step;
      r.newton_iterations = its;
      r.linear_iterations = st.linear_iterations;
      r.rejected = rejected;
      r.assemble_ms = st.assemble_ms;
      r.setup_ms = st.setup_ms;
      r.solve_ms = st.solve_ms;
      if (on_step) on_step(&r, *n_rec, user);
      ++*n_rec;
      rejected = 0;
      if (its < o->newton_desired)
        dd = std::min(dd * o->grow, o->dd_max);
      else if (its > o->newton_desired)
        dd = std::max(dd * o->shrink, o->dd_min);
    }
  }
  const int rr = set_rho(p, rho0);
  return rc ? rc : rr;
}

int mvpf_set_tuning(mvpf_problem* p, const char* key, int level, int value) {
  if (!p || !key || value < 0) return MVPF_EINVAL;
  p->config_version++;
  if (!std::strcmp(key, "row_blocks")) {
    if (level < 0 || level >= p->L) return MVPF_EINVAL;
    p->row_G[level] = value;
  } else if (!std::strcmp(key, "outer_blocks")) {
    p->outer_G = value;
  } else if (!std::strcmp(key, "small_grid_nodes")) {
    p->small_nodes = value;
  } else if (!std::strcmp(key, "coarse_overlap")) {
    p->coarse_overlap = value;
  } else if (!std::strcmp(key, "autotune_cache")) {
    if (value > 1) { p->err = "autotune_cache is 0 or 1"; return MVPF_EINVAL; }
    p->tune_cache_use = value;
  } else if (!std::strcmp(key, "mf_elements_per_block")) {
    if (value != 8 && value != 16 && value != 32) { p->err = "mf_elements_per_block is 8, 16 or 32"; return MVPF_EINVAL; }
    p->mf_epw = value;
  } else if (!std::strcmp(key, "assembly_slab_elements")) {
    // 0 = the allocated capacity; at least two element layers
    const int64_t lo = 2 * (int64_t)p->lev[0].g.nx * p->lev[0].g.ny + TILE;
    if (value != 0 && (value < lo || value > p->ne_cap)) {
      p->err = "assembly_slab_elements out of range";
      return MVPF_EINVAL;
    }
    p->ne_use = value == 0 ? p->ne_cap : value;
  } else if (!std::strcmp(key, "matrix_free")) {
    if (value > 1 || (value && p->L < 2)) { p->err = "matrix_free is 0 or 1 (and needs two levels)"; return MVPF_EINVAL; }
    if (value && !MF_AVAILABLE) { p->err = "the matrix-free finest level exists for six variants only"; return MVPF_EINVAL; }
    Level& L0 = p->lev[0];
    if (value && !p->Dmf64) {
      TRY(dalloc(p, &p->Dmf64, mf_hessian_values(L0.g)));
      if (p->mixed) TRY(dalloc(p, &p->Dmf32, mf_hessian_values(L0.g)));
    }
    if (value && p->mixed && !L0.DinvS32) TRY(dalloc(p, &L0.DinvS32, (size_t)L0.g.ntiles * LaySym<float>::SLICE));
    if (!value && !L0.A64) {  // the stored finest operator, on first use
      TRY(dalloc(p, &L0.A64, (size_t)L0.g.ntiles * NUP * Lay<double>::SLICE));
      if (p->mixed) TRY(dalloc(p, &L0.A32, (size_t)L0.g.ntiles * NUP * Lay<float>::SLICE));
    }
    p->mf = value;
    p->have_system = p->have_solution = false;  // the finest operator must be rebuilt
  } else {
    p->err = "unknown tuning key";
    return MVPF_EINVAL;
  }
  return 0;
}

int mvpf_get_tuning(const mvpf_problem* p, const char* key, int level, int* value) {
  if (!p || !key || !value) return MVPF_EINVAL;
  if (!std::strcmp(key, "row_blocks")) {
    if (level < 0 || level >= p->L) return MVPF_EINVAL;
    *value = p->row_G[level];
  } else if (!std::strcmp(key, "outer_blocks")) {
    *value = p->outer_G;
  } else if (!std::strcmp(key, "small_grid_nodes")) {
    *value = p->small_nodes;
  } else if (!std::strcmp(key, "assembly_slab_elements")) {
    *value = (int)p->ne_use;
  } else if (!std::strcmp(key, "matrix_free")) {
    *value = p->mf;
  } else if (!std::strcmp(key, "mf_elements_per_block")) {
    *value = p->mf_epw;
  } else if (!std::strcmp(key, "autotune_cache")) {
    *value = p->tune_cache_use;
  } else if (!std::strcmp(key, "coarse_overlap")) {
    const int nd = p->lev[p->L - 1].ndense;
    *value = p->coarse_overlap < 0 ? (nd <= COARSE_OVERLAP_MAX ? 1 : 0) : (p->coarse_overlap != 0);
  } else {
    return MVPF_EINVAL;
  }
  return 0;
}


int mvpf_autotune(mvpf_problem* p, int* row_blocks_out) {
  if (!p) return MVPF_EINVAL;
  p->config_version++;
  if (!p->have_system) { p->err = "autotune needs a Newton system"; return MVPF_ESTATE; }
  int tuned[MAX_LEVELS] = {0};
  if (p->mixed)
    autotune_levels<float>(p, tuned);
  else
    autotune_levels<double>(p, tuned);
  TRY(launch_check(p, "autotune"));
  if (row_blocks_out)
    for (int l = 0; l < p->L; ++l) row_blocks_out[l] = tuned[l];
  return 0;
}

int mvpf_kernel_timing(mvpf_problem* p, int enable) {
  if (!p) return MVPF_EINVAL;
  (void)hipStreamSynchronize(p->stream);
  for (KernelTimer* t : {&p->t_sweep, &p->t_outer, &p->t_resid, &p->t_qp}) {
    t->used = 0;
    t->launches = 0;
    t->total_ms = 0.0;
  }
  p->timing = enable != 0;
  return 0;
}

int mvpf_kernel_stats(mvpf_problem* p, const char* name, int* launches, double* total_ms, double* bytes_per_launch) {
  if (!p || !name) return MVPF_EINVAL;
  KernelTimer* t = nullptr;
  if (!std::strcmp(name, "pbj_sweep")) t = &p->t_sweep;
  else if (!std::strcmp(name, "spmv_outer")) t = &p->t_outer;
  else if (!std::strcmp(name, "residual")) t = &p->t_resid;
  else if (!std::strcmp(name, "qp_hessian")) t = &p->t_qp;
  else { p->err = "unknown kernel name"; return MVPF_EINVAL; }
  timer_collect(p, *t);
  if (launches) *launches = t->launches;
  if (total_ms) *total_ms = t->total_ms;
  if (bytes_per_launch) *bytes_per_launch = t->bytes;
  return 0;
}


// ---- batches ----------------------------------------------------------------

int mvpf_create_batch(int n, const mvpf_mesh* meshes, const mvpf_material* mats, const mvpf_loading* loads,
                      const mvpf_opts* opts, void* stream, mvpf_batch** out) {
  if (!out) return MVPF_EINVAL;
  *out = nullptr;
  if (n < 1 || n > MVPF_MAX_BATCH || !meshes || !mats || !loads || !opts) {
    g_create_err = "bad batch arguments";
    return MVPF_EINVAL;
  }
  if (opts->coarse != MVPF_COARSE_REDISCRETISE) {
    g_create_err = "batches use rediscretised coarse levels (opts.coarse = MVPF_COARSE_REDISCRETISE)";
    return MVPF_EINVAL;
  }
  mvpf_batch* b = new mvpf_batch();
  b->n = n;
  b->mixed = opts->precision == MVPF_MIXED;
  b->stream = (hipStream_t)stream;
  b->probs.assign(n, nullptr);
  b->vin.assign(n, nullptr);
  b->zout.assign(n, nullptr);
  b->branch.assign(n, nullptr);
  b->join.assign(n, nullptr);
  b->graph_version.assign(n, -1);
  int rc = 0;
  for (int i = 0; i < n && rc == 0; ++i) {
    rc = mvpf_create(&meshes[i], &mats[i], &loads[i], opts, stream, &b->probs[i]);
    if (rc) break;
    // a batched launch is wide even where each problem's level is small: the
    // two-pass kernels (every stored block read once) beat the small-grid
    // ones there (batched solve 336 -> 314 ms on the 32-problem workload)
    b->probs[i]->small_nodes = BATCH_SMALL_GRID_NODES;
    const int64_t nv = nvec(b->probs[i]->lev[0].g);
    if (hipMalloc((void**)&b->vin[i], sizeof(double) * nv) != hipSuccess ||
        hipMalloc(&b->zout[i], (b->mixed ? sizeof(float) : sizeof(double)) * nv) != hipSuccess ||
        hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) != hipSuccess) {
      g_create_err = "batch allocation failed";
      rc = MVPF_ENOMEM;
    }
  }
  if (rc == 0 && (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                  hipEventCreateWithFlags(&b->enter, hipEventDisableTiming) != hipSuccess ||
                  hipEventCreateWithFlags(&b->leave, hipEventDisableTiming) != hipSuccess ||
                  hipStreamCreateWithFlags(&b->work, hipStreamNonBlocking) != hipSuccess)) {
    g_create_err = "batch stream/event creation failed";
    rc = MVPF_EDEVICE;
  }
  if (rc == 0) {
    // job table of the batched coarse inversion (workspaces fixed per problem)
    std::vector<GJJob> tab(n);
    b->gj_n.resize(n);
    for (int i = 0; i < n; ++i) {
      mvpf_problem* p = b->probs[i];
      Level& C = p->lev[p->L - 1];
      const int nd = C.ndense;
      double* work = p->coarse_work ? p->coarse_work : p->V;
      tab[i] = gj_make_job(nd, work, C.Ainv, work + (int64_t)nd * nd, setup_status(p));
      b->gj_n[i] = nd;
    }
    const std::vector<int> sel = dense_invert_batch_selection(b->gj_n);
    if (hipMalloc((void**)&b->gj_tab, sizeof(GJJob) * n) != hipSuccess ||
        hipMalloc((void**)&b->gj_sel, sizeof(int) * n) != hipSuccess ||
        hipMemcpy(b->gj_tab, tab.data(), sizeof(GJJob) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->gj_sel, sel.data(), sizeof(int) * n, hipMemcpyHostToDevice) != hipSuccess) {
      g_create_err = "batch job tables failed";
      rc = MVPF_ENOMEM;
    }
  }
  if (rc) {
    batch_free(b);
    delete b;
    return rc;
  }
  *out = b;
  return 0;
}

void mvpf_destroy_batch(mvpf_batch* b) {
  if (!b) return;
  batch_free(b);
  delete b;
}

const char* mvpf_batch_last_error(const mvpf_batch* b) {
  if (!b) return g_create_err.c_str();
  return b->err.c_str();
}

mvpf_problem* mvpf_batch_problem(mvpf_batch* b, int i) {
  if (!b || i < 0 || i >= b->n) return nullptr;
  return b->probs[i];
}

// All problems' assembly and setup are enqueued before one synchronisation:
// batched launches on one stream when every level of every problem is a
// single slab, else each problem on its own branch stream; in both cases
// the coarsest-level inversions of all problems run as one batched chain.
int mvpf_batch_newton_system(mvpf_batch* b, const double* depths) {
  if (!b || !depths) return MVPF_EINVAL;
  for (mvpf_problem* p : b->probs)
    if (p->opts.coarse != MVPF_COARSE_REDISCRETISE) {
      b->err = "batches use rediscretised coarse levels (opts.coarse = MVPF_COARSE_REDISCRETISE)";
      return MVPF_EINVAL;
    }
  BCHK(hipEventRecord(b->enter, b->stream));
  int rc = 0, bad = -1;
  if (batch_single_slabs(b)) {
    // batched launches on one stream
    hipStream_t s = b->branch[0];
    BCHK(hipStreamWaitEvent(s, b->enter, 0));
    for (mvpf_problem* p : b->probs) {
      p->have_system = p->have_solution = false;
      p->stream = s;
    }
    rc = batch_assemble(b, depths, s);
    for (mvpf_problem* p : b->probs) p->stream = b->stream;
    (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(b->work);
    if (rc) return rc;
  } else {
    // largest coarsest levels first: their latency-bound inversions are the
    // longest chains and start while the other problems assemble
    std::vector<int> order(b->n);
    for (int i = 0; i < b->n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return b->probs[x]->lev[b->probs[x]->L - 1].ndense > b->probs[y]->lev[b->probs[y]->L - 1].ndense;
    });
    for (int oi = 0; oi < b->n && rc == 0; ++oi) {
      const int i = order[oi];
      mvpf_problem* p = b->probs[i];
      p->have_system = p->have_solution = false;
      BCHK(hipStreamWaitEvent(b->branch[i], b->enter, 0));
      p->stream = b->branch[i];
      rc = build_system(p, depths[i], false);
      p->stream = b->stream;
      if (rc) bad = i;
    }
    // all coarsest-level inversions at once, on the batch's work stream, after
    // every problem's dense coarse matrix is ready; each problem's setup waits
    if (rc == 0) {
      for (int i = 0; i < b->n; ++i) BCHK(hipStreamWaitEvent(b->work, b->probs[i]->ev_fork, 0));
      if (dense_invert_batch(b->gj_tab, b->gj_sel, b->gj_n, b->work) != 0) {
        b->err = "batched coarse inversion launch failed";
        rc = MVPF_EDEVICE;
      }
      for (int i = 0; i < b->n && rc == 0; ++i) BCHK(hipEventRecord(b->probs[i]->ev_join, b->work));
    }
    for (int oi = 0; oi < b->n && rc == 0; ++oi) {
      const int i = order[oi];
      mvpf_problem* p = b->probs[i];
      p->stream = b->branch[i];
      rc = setup_enqueue(p);
      p->stream = b->stream;
      if (rc) bad = i;
    }
    for (int i = 0; i < b->n; ++i) (void)hipStreamSynchronize(b->branch[i]);
    if (rc) {
      b->err = "problem " + std::to_string(bad) + ": " + b->probs[bad]->err;
      return rc;
    }
  }
  for (int i = 0; i < b->n; ++i) {
    mvpf_problem* p = b->probs[i];
    rc = setup_finish(p);
    if (rc) {
      b->err = "problem " + std::to_string(i) + ": " + p->err;
      return rc;
    }
    p->sys_depth = depths[i];
    p->have_system = true;
  }
  return 0;
}

int mvpf_batch_solve(mvpf_batch* b, mvpf_solve_stats* stats) {
  if (!b || !stats) return MVPF_EINVAL;
  for (int i = 0; i < b->n; ++i)
    if (!b->probs[i]->have_system) {
      b->err = "problem " + std::to_string(i) + " has no Newton system";
      return MVPF_ESTATE;
    }
  BCHK(hipStreamSynchronize(b->stream));  // the caller's pending work (states, systems)
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < b->n; ++i) b->probs[i]->stream = b->work;
  int rc = b->mixed ? batch_fgmres<float, float>(b, stats) : batch_fgmres<double, double>(b, stats);
  for (int i = 0; i < b->n; ++i) {
    b->probs[i]->stream = b->stream;
    (void)hipStreamSynchronize(b->branch[i]);
  }
  (void)hipStreamSynchronize(b->work);
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rc < 0) {
    if (b->err.empty()) b->err = "batched solve failed";
    return rc;
  }
  for (int i = 0; i < b->n; ++i) {
    stats[i].solve_ms = ms;
    b->probs[i]->have_solution = true;
  }
  if (rc == MVPF_ENOTCONV) b->err = "FGMRES reached max_it on at least one problem";
  return rc;
}

int mvpf_batch_newton_update(mvpf_batch* b) {
  if (!b) return MVPF_EINVAL;
  for (int i = 0; i < b->n; ++i) {
    const int rc = mvpf_newton_update(b->probs[i]);
    if (rc) {
      b->err = "problem " + std::to_string(i) + ": " + b->probs[i]->err;
      return rc;
    }
  }
  return 0;
}

}  // extern "C"
