// Local (quadrature-point) derivatives of the penalised incremental potential
// density with respect to q = (F_00..F_22 row-major, eta_1..eta_N).
//
// Density (Sec. 2.2-2.3, 3.1-3.2; gradient-energy part handled separately by
// the element kernels since it is a constant quadratic form):
//   psi = sum_i eta_i F_i + 1/2 J_t H : L(eta) H + sum_{i<j} w_ij eta_i eta_j
//         + sum_i rho/2 (eta_i - eta_in)^2 + sum_i eps/2 <eta_i>_-^2
//   F^t = I + sum_k eta_k dU_k  (Eq. LinMix with U_0 = I, condensed),
//   J_t = det F^t, G = (F^t)^-1, C = G F^T F G  (C^e of Eq. elasticEn),
//   H = A(C) B(C)^-1, the Pade approximant of 1/2 log C of order (1,1), (2,2)
//   or (3,3) (Eqs. pade11, pade22, pade33; A and B are matrix polynomials in
//   C, the leading factor folded into A), L = L_0 + sum eta_k dL_k.
//
// Derivatives are closed-form:
//  * in C-space along the symmetric basis E_v (xx,yy,zz,yz,xz,xy; the shear
//    ones are e_a e_b^T + e_b e_a^T); A, B commute with C, so with
//    dX_v = dX/dC[E_v] and d2X_uv its second derivative (X = A, B):
//    dH = (dA - H dB) B^-1,
//    d2H = (d2A - dH_u dB_v - dH_v dB_u - H d2B) B^-1, where
//    d(C^2)[E] = CE + EC, d(C^3)[E] = EC^2 + CEC + C^2E,
//    d2(C^2)[E_u, E_v] = E_u E_v + E_v E_u,
//    d2(C^3)[E_u, E_v] = (E_u E_v + E_v E_u) C + C (E_u E_v + E_v E_u) + E_u C E_v + E_v C E_u;
//  * chain rule through C(F, G(eta)), J_t(eta), L(eta):
//    dC/dF_ij = a_i (x) G_j + G_j (x) a_i  (a_i = row i of F G),
//    dC/deta_k = -(Q_k C + C Q_k^T), Q_k = G dU_k,  dJ_t/deta_k = J_t tr Q_k,
//    d2C/dF_ij dF_kl = delta_ik (G_j (x) G_l + G_l (x) G_j),
//    d2C/dF deta_k = -(Q_k dC_F + dC_F Q_k^T),
//    d2C/deta_k deta_l = sym2(Q_k Q_l C + Q_l Q_k C + Q_k C Q_l^T),
//    d2J_t/deta_k deta_l = J_t (tr Q_k tr Q_l - tr(Q_k Q_l)).
#pragma once
#include <hip/hip_runtime.h>

// Number of martensite variants N: a compile-time constant of the library
// (each build is one instantiation; 6 for CuAlNi, Sec. 4.1; 12 for a
// NiTi-like card, the footnote of Sec. 4.4).
#ifndef MVPF_NVAR
#define MVPF_NVAR 6
#endif

namespace mvpf {

constexpr int NV = MVPF_NVAR;           // variants N (order parameters per node)
constexpr int NQ = 9 + NV;              // local variables of a Gauss point: F (9), eta_hat (N)
constexpr int NHP = NQ * (NQ + 1) / 2;  // packed upper triangle of their Hessian
static_assert(NV >= 1 && NV <= 13, "unknowns per node must fit the 16-bit constraint masks");

// Material card on the device, in the sample frame.
struct DevCard {
  double dU[NV][6];    // U_k - I (k = 1..N) as symmetric components
  double L0[6][6];     // austenite stiffness, Voigt (engineering shear strain)
  double dL[NV][6][6];  // L_k - L_0
  double dF0[NV];      // F_k - F_0
  double W[NV + 1][NV + 1];   // double-obstacle coefficients, zero diagonal
  double Sw[NV][NV];     // condensed Hessian of 1/2 eta^T W eta w.r.t. eta_hat
  double Mg[NV][NV];     // gradient-energy species matrix: psi_g = 1/2 Mg_kl grad eta_k . grad eta_l
  float Mg32[NV][NV];    // Mg rounded to FP32 (the FP32 matrix-free operator)
  double rho;
  double eps;
  int pade;
  int mixing;          // MVPF_MIX_LINEAR (Eq. LinMix) or MVPF_MIX_LOG
  double logU[NV][6];  // log U_k (logarithmic mixing rule, Sec. 2.1)
};

// symmetric index map (xx,yy,zz,yz,xz,xy)
__host__ __device__ constexpr int SI(int a, int b) {
  return a == b ? a : (a + b == 3 ? 3 : (a + b == 2 ? 4 : 5));
}

__device__ __forceinline__ void full_from_sym(const double s[6], double m[9]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) m[3 * a + b] = s[SI(a, b)];
}

// symmetric part components of a full matrix
__device__ __forceinline__ void sym_of(const double m[9], double s[6]) {
  s[0] = m[0];
  s[1] = m[4];
  s[2] = m[8];
  s[3] = 0.5 * (m[5] + m[7]);
  s[4] = 0.5 * (m[2] + m[6]);
  s[5] = 0.5 * (m[1] + m[3]);
}

__device__ __forceinline__ void mm(const double a[9], const double b[9], double c[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

__device__ __forceinline__ double ddot9(const double a[9], const double b[9]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) s += a[i] * b[i];
  return s;
}

// sum_ab a_ab b_ba
__device__ __forceinline__ double trprod(const double a[9], const double b[9]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s += a[3 * i + j] * b[3 * j + i];
  return s;
}

// Contraction X : E_v of a full matrix with the symmetric basis element E_v.
__device__ __forceinline__ double contract_basis(const double x[9], int v) {
  switch (v) {
    case 0: return x[0];
    case 1: return x[4];
    case 2: return x[8];
    case 3: return x[5] + x[7];
    case 4: return x[2] + x[6];
    default: return x[1] + x[3];
  }
}

// engineering (Voigt strain) form of symmetric components
__device__ __forceinline__ void eng(const double s[6], double e[6]) {
  e[0] = s[0]; e[1] = s[1]; e[2] = s[2];
  e[3] = 2.0 * s[3]; e[4] = 2.0 * s[4]; e[5] = 2.0 * s[5];
}

// inverse and determinant of a symmetric 3x3 (components)
__device__ __forceinline__ double sym_inv(const double s[6], double r[6]) {
  const double xx = s[0], yy = s[1], zz = s[2], yz = s[3], xz = s[4], xy = s[5];
  const double c0 = yy * zz - yz * yz;
  const double c5 = xz * yz - xy * zz;  // cofactor (0,1)
  const double c4 = xy * yz - xz * yy;  // cofactor (0,2)
  const double det = xx * c0 + xy * c5 + xz * c4;
  const double id = 1.0 / det;
  r[0] = c0 * id;
  r[5] = c5 * id;
  r[4] = c4 * id;
  r[1] = (xx * zz - xz * xz) * id;
  r[3] = (xy * xz - xx * yz) * id;
  r[2] = (xx * yy - xy * xy) * id;
  return det;
}

// Symmetric basis element E_v as a full matrix.
__device__ __forceinline__ void basis(int v, double e[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) e[i] = 0.0;
  switch (v) {
    case 0: e[0] = 1.0; break;
    case 1: e[4] = 1.0; break;
    case 2: e[8] = 1.0; break;
    case 3: e[5] = e[7] = 1.0; break;
    case 4: e[2] = e[6] = 1.0; break;
    default: e[1] = e[3] = 1.0; break;
  }
}

__host__ __device__ constexpr int hidx(int p, int q) {  // packed upper triangle, p <= q < NQ
  return p * NQ - (p * (p - 1)) / 2 + (q - p);
}

// Coefficients of H = A B^-1 with A = sum_p a_p C^p, B = sum_p b_p C^p.
template <int ORDER> struct Pade;
template <> struct Pade<11> {  // (C - I)(C + I)^-1
  static constexpr int deg = 1;
  __host__ __device__ static constexpr double a(int p) { return p == 0 ? -1.0 : (p == 1 ? 1.0 : 0.0); }
  __host__ __device__ static constexpr double b(int p) { return p <= 1 ? 1.0 : 0.0; }
};
template <> struct Pade<22> {  // 3/2 (C^2 - I)(C^2 + 4C + I)^-1
  static constexpr int deg = 2;
  __host__ __device__ static constexpr double a(int p) { return p == 0 ? -1.5 : (p == 2 ? 1.5 : 0.0); }
  __host__ __device__ static constexpr double b(int p) { return p == 1 ? 4.0 : (p <= 2 ? 1.0 : 0.0); }
};
template <> struct Pade<33> {  // 1/6 (11C^3 + 27C^2 - 27C - 11I)(C^3 + 9C^2 + 9C + I)^-1
  static constexpr int deg = 3;
  __host__ __device__ static constexpr double a(int p) {
    return p == 0 ? -11.0 / 6.0 : (p == 1 ? -4.5 : (p == 2 ? 4.5 : 11.0 / 6.0));
  }
  __host__ __device__ static constexpr double b(int p) { return (p == 0 || p == 3) ? 1.0 : 9.0; }
};

// x += c m, the term dropped at compile time when c is zero
template <int N>
__device__ __forceinline__ void axpy_c(double c, const double m[N], double x[N]) {
  if (c == 0.0) return;
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += c * m[i];
}

// Quantities shared by the gradient and the Hessian.
struct LocalBase {
  double Jt;
  double G[9];    // (F^t)^-1, full
  double Fe[9];   // F G
  double C[9];    // full symmetric
  double w;       // 1/2 H : L H
  double wC[6];   // dw/dC along E_v
  double wEta[NV]; // partial dw/deta_k at fixed C
  double dh[6][6];  // engineering components of dH_v
  double h[6];      // engineering H
  double T[6];      // L H (tensor components)
  double Binv[9];
  double H[9];
};

// With the logarithmic mixing rule F^t depends nonlinearly on eta: its
// first derivatives dF^t/deta_k are kept per Gauss point.
struct LocalBaseLog : LocalBase {
  double dFt[NV][6];  // dF^t / deta_k (symmetric components)
};
template <int MIX> struct BaseOf { using type = LocalBase; };
template <> struct BaseOf<1> { using type = LocalBaseLog; };

// dF^t / deta_k: the constant U_k - I (Eq. LinMix) or the stored derivative
__device__ __forceinline__ const double* dFt_of(const LocalBase& b, const DevCard& cd, int k) { return cd.dU[k]; }
__device__ __forceinline__ const double* dFt_of(const LocalBaseLog& b, const DevCard& cd, int k) { return b.dFt[k]; }

// Terms of the power series of exp: exact to rounding for ||M||_F <= 1
// (the omitted tail is below 1/19! ~ 8e-18 there; the order parameters of
// the workloads keep ||sum eta_k log U_k|| near 0.1).
constexpr int EXP_TERMS = 18;

__device__ __forceinline__ void log_mixing_matrix(const double eh[NV], const DevCard& cd, double M[9]) {
  double Ms[6];
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) s += eh[k] * cd.logU[k][v];
    Ms[v] = s;
  }
  full_from_sym(Ms, M);
}

// F^t = exp(M), M = sum_k eta_k log U_k (logarithmic mixing, Sec. 2.1), and
// dF^t/deta_k = sum_n 1/n! d(M^n)[log U_k], by the power series with the
// recurrences M^n = M^(n-1) M and d(M^n)[A] = d(M^(n-1))[A] M + M^(n-1) A.
__device__ __forceinline__ void log_mixing(const double eh[NV], const DevCard& cd, double Ft[6],
                                           double dFt[NV][6]) {
  double M[9], P[9], E[9];
  log_mixing_matrix(eh, cd, M);
  double D[NV][9], Sd[NV][9];
#pragma unroll
  for (int i = 0; i < 9; ++i) P[i] = E[i] = (i % 4 == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int i = 0; i < 9; ++i) D[k][i] = Sd[k][i] = 0.0;
  double c = 1.0;
#pragma unroll 1
  for (int n = 1; n <= EXP_TERMS; ++n) {
    c /= n;
    double T[9];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double A[9], DM[9], PA[9];
      full_from_sym(cd.logU[k], A);
      mm(D[k], M, DM);
      mm(P, A, PA);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        D[k][i] = DM[i] + PA[i];
        Sd[k][i] += c * D[k][i];
      }
    }
    mm(P, M, T);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      P[i] = T[i];
      E[i] += c * P[i];
    }
  }
  sym_of(E, Ft);
#pragma unroll
  for (int k = 0; k < NV; ++k) sym_of(Sd[k], dFt[k]);
}

// d^2 F^t / deta_k deta_l = sum_n 1/n! d^2(M^n)[A_k, A_l] (A = log U) with
// d^2(M^n)[A_k, A_l] = d^2(M^(n-1))[A_k, A_l] M + d(M^(n-1))[A_l] A_k
//                      + d(M^(n-1))[A_k] A_l.
__device__ __forceinline__ void log_mixing_second(const double eh[NV], const DevCard& cd, int k, int l,
                                                  double out[9]) {
  double M[9], P[9], Dk[9], Dl[9], S[9], Ak[9], Al[9];
  log_mixing_matrix(eh, cd, M);
  full_from_sym(cd.logU[k], Ak);
  full_from_sym(cd.logU[l], Al);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    P[i] = (i % 4 == 0) ? 1.0 : 0.0;
    Dk[i] = Dl[i] = S[i] = out[i] = 0.0;
  }
  double c = 1.0;
#pragma unroll 1
  for (int n = 1; n <= EXP_TERMS; ++n) {
    c /= n;
    double SM[9], DlA[9], DkA[9], DkM[9], DlM[9], PAk[9], PAl[9], T[9];
    mm(S, M, SM);
    mm(Dl, Ak, DlA);
    mm(Dk, Al, DkA);
    mm(Dk, M, DkM);
    mm(Dl, M, DlM);
    mm(P, Ak, PAk);
    mm(P, Al, PAl);
    mm(P, M, T);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      S[i] = SM[i] + DlA[i] + DkA[i];
      Dk[i] = DkM[i] + PAk[i];
      Dl[i] = DlM[i] + PAl[i];
      P[i] = T[i];
      out[i] += c * S[i];
    }
  }
}

// Hencky energy (Pade order PD) and its first C-derivatives; MIX: the
// mixing rule of F^t (0: Eq. LinMix, 1: logarithmic).
template <int PD, int MIX = 0>
__device__ __forceinline__ void local_base(const double F[9], const double eh[NV], const DevCard& cd,
                                           typename BaseOf<MIX>::type& b) {
  using P = Pade<PD>;
  double Ft[6];
  if constexpr (MIX == 1) {
    log_mixing(eh, cd, Ft, b.dFt);
  } else {
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      double s = (v < 3) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) s += eh[k] * cd.dU[k][v];
      Ft[v] = s;
    }
  }
  double Gs[6];
  b.Jt = sym_inv(Ft, Gs);
  full_from_sym(Gs, b.G);
  mm(F, b.G, b.Fe);
  // C = Fe^T Fe
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      b.C[3 * a + c] = b.Fe[a] * b.Fe[c] + b.Fe[3 + a] * b.Fe[3 + c] + b.Fe[6 + a] * b.Fe[6 + c];
  double C2[9], C3[9];
  if constexpr (P::deg >= 2) mm(b.C, b.C, C2);
  if constexpr (P::deg >= 3) mm(C2, b.C, C3);
  double Am[9], Bf[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double id = (i % 4 == 0) ? 1.0 : 0.0;
    Am[i] = P::a(0) * id + P::a(1) * b.C[i];
    Bf[i] = P::b(0) * id + P::b(1) * b.C[i];
  }
  if constexpr (P::deg >= 2) {
    axpy_c<9>(P::a(2), C2, Am);
    axpy_c<9>(P::b(2), C2, Bf);
  }
  if constexpr (P::deg >= 3) {
    axpy_c<9>(P::a(3), C3, Am);
    axpy_c<9>(P::b(3), C3, Bf);
  }
  double Bs[6], Bi[6];
  sym_of(Bf, Bs);
  sym_inv(Bs, Bi);
  full_from_sym(Bi, b.Binv);
  double Hf[9];
  mm(Am, b.Binv, Hf);
  double Hs[6];
  sym_of(Hf, Hs);
  full_from_sym(Hs, b.H);
  eng(Hs, b.h);
  // mixed stiffness and Hencky stress
  double Lm[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double s = cd.L0[i][j];
#pragma unroll
      for (int k = 0; k < NV; ++k) s += eh[k] * cd.dL[k][i][j];
      Lm[i][j] = s;
    }
  double w = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) s += Lm[i][j] * b.h[j];
    b.T[i] = s;
    w += b.h[i] * s;
  }
  b.w = 0.5 * w;
  // partial derivative w.r.t. eta at fixed C: 1/2 h^T dL_k h
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) t += cd.dL[k][i][j] * b.h[j];
      s += b.h[i] * t;
    }
    b.wEta[k] = 0.5 * s;
  }
  // dH along the C basis and dw/dC
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    double E[9], dA[9], dB[9], HdB[9], X[9], dHf[9], dHs[6];
    basis(v, E);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      dA[i] = P::a(1) * E[i];
      dB[i] = P::b(1) * E[i];
    }
    if constexpr (P::deg >= 2) {
      double CE[9], d2[9];
      mm(b.C, E, CE);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) d2[3 * a + c] = CE[3 * a + c] + CE[3 * c + a];
      axpy_c<9>(P::a(2), d2, dA);
      axpy_c<9>(P::b(2), d2, dB);
      if constexpr (P::deg >= 3) {
        double C2E[9], CEC[9], d3[9];
        mm(C2, E, C2E);
        mm(CE, b.C, CEC);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) d3[3 * a + c] = C2E[3 * a + c] + C2E[3 * c + a] + CEC[3 * a + c];
        axpy_c<9>(P::a(3), d3, dA);
        axpy_c<9>(P::b(3), d3, dB);
      }
    }
    mm(b.H, dB, HdB);
#pragma unroll
    for (int i = 0; i < 9; ++i) X[i] = dA[i] - HdB[i];
    mm(X, b.Binv, dHf);
    sym_of(dHf, dHs);
    eng(dHs, b.dh[v]);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) s += b.T[i] * b.dh[v][i];
    b.wC[v] = s;
  }
}

// Symmetric components of dC along variable q (0..8: F_ij row-major; 9..: eta).
template <class B>
__device__ __forceinline__ void dC_of(const B& b, const DevCard& cd, int q, double dc[6], double dcf[9]) {
  if (q < 9) {
    const int i = q / 3, j = q % 3;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        dcf[3 * a + c] = b.Fe[3 * i + a] * b.G[3 * c + j] + b.G[3 * a + j] * b.Fe[3 * i + c];
  } else {
    const int k = q - 9;
    double dU[9], Q[9], X[9];
    full_from_sym(dFt_of(b, cd, k), dU);
    mm(b.G, dU, Q);
    mm(Q, b.C, X);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) dcf[3 * a + c] = -(X[3 * a + c] + X[3 * c + a]);
  }
  dc[0] = dcf[0]; dc[1] = dcf[4]; dc[2] = dcf[8];
  dc[3] = dcf[5]; dc[4] = dcf[2]; dc[5] = dcf[1];
}

// a[i] for a runtime i in 0..N-1 (selection, no indexing: the array stays
// in registers)
__device__ __forceinline__ double pick6(int i, double a0, double a1, double a2, double a3, double a4, double a5) {
  double r = a0;
  r = (i == 1) ? a1 : r;
  r = (i == 2) ? a2 : r;
  r = (i == 3) ? a3 : r;
  r = (i == 4) ? a4 : r;
  r = (i == 5) ? a5 : r;
  return r;
}
// a[i] of the N values at a (same selection chain)
template <int N>
__device__ __forceinline__ double pick_n(int i, const double* a) {
  if constexpr (N == 6) {
    return pick6(i, a[0], a[1], a[2], a[3], a[4], a[5]);
  } else {
    double r = a[0];
#pragma unroll
    for (int j = 1; j < N; ++j) r = (i == j) ? a[j] : r;
    return r;
  }
}
template <int N>
__device__ __forceinline__ double pick(int i, const double (&a)[N]) {
  if constexpr (N == 6) {
    return pick6(i, a[0], a[1], a[2], a[3], a[4], a[5]);
  } else {
    double r = a[0];
#pragma unroll
    for (int j = 1; j < N; ++j) r = (i == j) ? a[j] : r;
    return r;
  }
}
// a[i][v] for a runtime i (selection, as pick)
template <int N, int M>
__device__ __forceinline__ double pick_row(int i, const double (&a)[N][M], int v) {
  if constexpr (N == 6) {
    return pick6(i, a[0][v], a[1][v], a[2][v], a[3][v], a[4][v], a[5][v]);
  } else {
    double r = a[0][v];
#pragma unroll
    for (int j = 1; j < N; ++j) r = (i == j) ? a[j][v] : r;
    return r;
  }
}

// Q_k = G dF^t/deta_k (full)
template <class B>
__device__ __forceinline__ void Q_of(const B& b, const DevCard& cd, int k, double Q[9]) {
  double dU[9];
  full_from_sym(dFt_of(b, cd, k), dU);
  mm(b.G, dU, Q);
}

// dC/deta_k = -(Q_k C + C Q_k^T) as symmetric components (and full)
__device__ __forceinline__ void dC_eta(const LocalBase& b, const double Q[9], double dc[6], double dcf[9]) {
  double X[9];
  mm(Q, b.C, X);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) dcf[3 * a + c] = -(X[3 * a + c] + X[3 * c + a]);
  dc[0] = dcf[0]; dc[1] = dcf[4]; dc[2] = dcf[8];
  dc[3] = dcf[5]; dc[4] = dcf[2]; dc[5] = dcf[1];
}

// dC/dF_ij (q = 3 i + j) as symmetric components
__device__ __forceinline__ void dC_F(const LocalBase& b, int q, double dc[6]) {
  const int i = q / 3, j = q % 3;
  // dcf[a][c] = Fe[i][a] G[c][j] + G[a][j] Fe[i][c]
  auto f = [&](int a, int c) { return b.Fe[3 * i + a] * b.G[3 * c + j] + b.G[3 * a + j] * b.Fe[3 * i + c]; };
  dc[0] = f(0, 0); dc[1] = f(1, 1); dc[2] = f(2, 2);
  dc[3] = f(1, 2); dc[4] = f(0, 2); dc[5] = f(0, 1);
}

__device__ __forceinline__ double neg_part(double x) { return x < 0.0 ? x : 0.0; }

// Gradient of the local density: g[NQ].
template <int PD, int MIX = 0>
__device__ __forceinline__ void local_gradient(const double F[9], const double eh[NV], const double ehn[NV],
                                               const DevCard& cd, double g[NQ]) {
  typename BaseOf<MIX>::type b;
  local_base<PD, MIX>(F, eh, cd, b);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double dc[6], dcf[9];
    dC_of(b, cd, q, dc, dcf);
    double wq = 0.0;
#pragma unroll
    for (int v = 0; v < 6; ++v) wq += b.wC[v] * dc[v];
    if (q < 9) {
      g[q] = b.Jt * wq;
    } else {
      const int k = q - 9;
      double dU[9], Q[9];
      full_from_sym(dFt_of(b, cd, k), dU);
      mm(b.G, dU, Q);
      const double trQ = Q[0] + Q[4] + Q[8];
      g[q] = b.Jt * (wq + b.wEta[k]) + b.Jt * trQ * b.w;
    }
  }
  // order-parameter terms: chemical, double obstacle, viscous, penalty
  double eta[NV + 1], etan[NV + 1];
  double s = 0.0, sn = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) { eta[k + 1] = eh[k]; etan[k + 1] = ehn[k]; s += eh[k]; sn += ehn[k]; }
  eta[0] = 1.0 - s;
  etan[0] = 1.0 - sn;
  double We[NV + 1];
#pragma unroll
  for (int i = 0; i < NV + 1; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < NV + 1; ++j) t += cd.W[i][j] * eta[j];
    We[i] = t;
  }
  const double d0 = eta[0] - etan[0];
  const double n0 = neg_part(eta[0]);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    g[9 + k] += cd.dF0[k] + (We[k + 1] - We[0]) + cd.rho * ((eta[k + 1] - etan[k + 1]) - d0)
                + cd.eps * (neg_part(eta[k + 1]) - n0);
  }
}

// Gradient and packed upper-triangular Hessian of the local density; entry
// hidx(p, q) of the Hessian is stored to D[hidx(p, q) * ds] as soon as it is
// known (nothing of it is kept in registers).
template <int PD, int MIX = 0>
__device__ __forceinline__ void local_hessian(const double F[9], const double eh[NV], const double ehn[NV],
                                              const DevCard& cd, double g[NQ], double* __restrict__ D,
                                              int64_t ds) {
  using P = Pade<PD>;
  typename BaseOf<MIX>::type b;
  local_base<PD, MIX>(F, eh, cd, b);
  // ---- second derivatives in C-space -------------------------------------
  double wCC[6][6];
  double wCeta[6][NV];  // [v][k]
  {
    double Lm[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double s = cd.L0[i][j];
#pragma unroll
        for (int k = 0; k < NV; ++k) s += eh[k] * cd.dL[k][i][j];
        Lm[i][j] = s;
      }
    // T : d2H_uv = Y : (d2A - H d2B) - V_u : dB_v - V_v : dB_u with Y = T B^-1,
    // V_u = dH_u Y.  Y : (d2A - H d2B) = Zt : (E_u E_v + E_v E_u)
    // + Z_3 : (E_u C E_v + E_v C E_u) with Z_p = a_p Y - b_p H Y and
    // Zt = Z_2 + Z_3 C + C Z_3;  V : dB_v = Vt : E_v with
    // Vt = b_1 V + b_2 (CV + VC) + b_3 (V C^2 + C V C + C^2 V).
    double Tf[9], Ts[6] = {b.T[0], b.T[1], b.T[2], b.T[3], b.T[4], b.T[5]};
    full_from_sym(Ts, Tf);
    double Y[9], HY[9], Zt[9], Z3[9], C2[9];
    mm(Tf, b.Binv, Y);
    mm(b.H, Y, HY);
    if constexpr (P::deg >= 2) {
#pragma unroll
      for (int i = 0; i < 9; ++i) Zt[i] = P::a(2) * Y[i] - P::b(2) * HY[i];
    }
    if constexpr (P::deg >= 3) {
      double ZC[9], CZ[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) Z3[i] = P::a(3) * Y[i] - P::b(3) * HY[i];
      mm(Z3, b.C, ZC);
      mm(b.C, Z3, CZ);
#pragma unroll
      for (int i = 0; i < 9; ++i) Zt[i] += ZC[i] + CZ[i];
      mm(b.C, b.C, C2);
    }
    double vt[6][6];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      double dHs[6] = {b.dh[u][0], b.dh[u][1], b.dh[u][2],
                       0.5 * b.dh[u][3], 0.5 * b.dh[u][4], 0.5 * b.dh[u][5]};
      double dHf[9], V[9], Vt[9];
      full_from_sym(dHs, dHf);
      mm(dHf, Y, V);
#pragma unroll
      for (int i = 0; i < 9; ++i) Vt[i] = P::b(1) * V[i];
      if constexpr (P::deg >= 2) {
        double CV[9], VC[9];
        mm(b.C, V, CV);
        mm(V, b.C, VC);
#pragma unroll
        for (int i = 0; i < 9; ++i) Vt[i] += P::b(2) * (CV[i] + VC[i]);
        if constexpr (P::deg >= 3) {
          double VC2[9], CVC[9], C2V[9];
          mm(V, C2, VC2);
          mm(CV, b.C, CVC);
          mm(C2, V, C2V);
#pragma unroll
          for (int i = 0; i < 9; ++i) Vt[i] += P::b(3) * (VC2[i] + CVC[i] + C2V[i]);
        }
      }
#pragma unroll
      for (int v = 0; v < 6; ++v) vt[u][v] = contract_basis(Vt, v);
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      double LdH[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += Lm[i][j] * b.dh[u][j];
        LdH[i] = s;
      }
#pragma unroll
      for (int v = 0; v <= u; ++v) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) s += b.dh[v][i] * LdH[i];
        double zd = 0.0;
        if constexpr (P::deg >= 2) {
          double Eu[9], Ev[9], P1[9], P2[9];
          basis(u, Eu);
          basis(v, Ev);
          mm(Eu, Ev, P1);
          mm(Ev, Eu, P2);
#pragma unroll
          for (int i = 0; i < 9; ++i) zd += Zt[i] * (P1[i] + P2[i]);
          if constexpr (P::deg >= 3) {
            double EC[9], ECE1[9], ECE2[9];
            mm(Eu, b.C, EC);
            mm(EC, Ev, ECE1);
            mm(Ev, b.C, EC);
            mm(EC, Eu, ECE2);
#pragma unroll
            for (int i = 0; i < 9; ++i) zd += Z3[i] * (ECE1[i] + ECE2[i]);
          }
        }
        const double val = s + zd - vt[u][v] - vt[v][u];
        wCC[u][v] = val;
        wCC[v][u] = val;
      }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double dLh[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += cd.dL[k][i][j] * b.h[j];
        dLh[i] = s;
      }
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) s += dLh[i] * b.dh[v][i];
        wCeta[v][k] = s;
      }
    }
  }
  // ---- chain rule ---------------------------------------------------------
  // Few arrays stay live: dC along F is rebuilt from F G and G when needed,
  // Q_k = G dU_k from the card, and the eta-eta products pair by pair.
  // S: symmetric tensor with S : dC = sum_v wC_v dc_v
  double Sf[9];
  {
    double Ss[6] = {b.wC[0], b.wC[1], b.wC[2], 0.5 * b.wC[3], 0.5 * b.wC[4], 0.5 * b.wC[5]};
    full_from_sym(Ss, Sf);
  }
  double GSG[9];
  {
    double GS[9];
    mm(b.G, Sf, GS);
    mm(GS, b.G, GSG);
  }
  // per eta_k: dC (dce), dw/deta_k (wqe), dJ_t (Jq)
  double dce[NV][6], wqe[NV], Jq[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double Q[9], dcf[9];
    Q_of(b, cd, k, Q);
    Jq[k] = b.Jt * (Q[0] + Q[4] + Q[8]);
    dC_eta(b, Q, dce[k], dcf);
    double s = b.wEta[k];
#pragma unroll
    for (int v = 0; v < 6; ++v) s += b.wC[v] * dce[k][v];
    wqe[k] = s;
    g[9 + k] = b.Jt * wqe[k] + Jq[k] * b.w;
  }
  // eta-eta block
  double eta[NV + 1], etan[NV + 1];
  {
    double s = 0.0, sn = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) { eta[k + 1] = eh[k]; etan[k + 1] = ehn[k]; s += eh[k]; sn += ehn[k]; }
    eta[0] = 1.0 - s;
    etan[0] = 1.0 - sn;
  }
  const double pen0 = (eta[0] < 0.0) ? cd.eps : 0.0;
  // Runtime (not unrolled) loops over the pairs k <= l: unrolled, the
  // compiler keeps every Q_l product of all pairs live at once.  Values of
  // the per-eta register arrays are picked by static-index selection.
#pragma unroll 1
  for (int k = 0; k < NV; ++k) {
    double Qk[9], SQ[9], Rk[9], Uk[9], WCk[6], dk[6], wek[6];
    Q_of(b, cd, k, Qk);
    mm(Sf, Qk, SQ);
    mm(b.C, SQ, Rk);  // C S Q_k
    mm(SQ, b.C, Uk);  // S Q_k C
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      dk[v] = pick_row(k, dce, v);
      wek[v] = pick(k, wCeta[v]);
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < 6; ++v) s += wCC[u][v] * dk[v];
      WCk[u] = s;
    }
    const double trk = Qk[0] + Qk[4] + Qk[8];
    const double Jqk = pick(k, Jq);
    const double wqk = pick(k, wqe);
    const double etak = pick_n<NV>(k, eta + 1);
#pragma unroll 1
    for (int l = k; l < NV; ++l) {
      double Ql[9], SQl[9], Rl[9], dl[6], wel[6];
      Q_of(b, cd, l, Ql);
      mm(Sf, Ql, SQl);
      mm(b.C, SQl, Rl);  // C S Q_l
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        dl[v] = pick_row(l, dce, v);
        wel[v] = pick(l, wCeta[v]);
      }
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < 6; ++u) s += WCk[u] * dl[u];
      s += 2.0 * (trprod(Rk, Ql) + trprod(Rl, Qk) + ddot9(Uk, Ql));
#pragma unroll
      for (int v = 0; v < 6; ++v) s += wel[v] * dk[v] + wek[v] * dl[v];
      const double trl = Ql[0] + Ql[4] + Ql[8];
      const double Jkl = b.Jt * (trk * trl - trprod(Qk, Ql));
      const double Jql = pick(l, Jq);
      const double wql = pick(l, wqe);
      double val = b.Jt * s + Jqk * wql + Jql * wqk + Jkl * b.w;
      if constexpr (MIX == 1) {
        // second derivative of F^t (nonzero under logarithmic mixing):
        // d2C gains -(Q_kl C + C Q_kl^T) and d2J_t gains J_t tr Q_kl, with
        // Q_kl = G d2F^t/deta_k deta_l
        double S2[9], Qkl[9], dckl[6], dcfkl[9];
        log_mixing_second(eh, cd, k, l, S2);
        mm(b.G, S2, Qkl);
        dC_eta(b, Qkl, dckl, dcfkl);
        double wkl = 0.0;
#pragma unroll
        for (int v = 0; v < 6; ++v) wkl += b.wC[v] * dckl[v];
        val += b.Jt * (wkl + (Qkl[0] + Qkl[4] + Qkl[8]) * b.w);
      }
      // order-parameter terms
      val += cd.Sw[k][l] + cd.rho * ((k == l ? 1.0 : 0.0) + 1.0) + pen0;
      if (k == l && etak < 0.0) val += cd.eps;
      D[hidx(9 + k, 9 + l) * ds] = val;
    }
  }
  // F-eta block, runtime loop over k: with ak = wCeta[., k] - 2 (S Q_k) : E_.
  // and wdk = wCC dC_k (wCC symmetric), entry (F_q, eta_k) is
  // J_t (wdk + ak) . dC_q + dJ_t/deta_k  dw/dF_q
#pragma unroll 1
  for (int k = 0; k < NV; ++k) {
    double Q[9], P[9], t[6];
    Q_of(b, cd, k, Q);
    mm(Sf, Q, P);  // S G dU_k
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      double wdk = 0.0;
#pragma unroll
      for (int v = 0; v < 6; ++v)
        wdk += wCC[u][v] * pick_row(k, dce, v);
      t[u] = wdk + pick(k, wCeta[u]) -
             2.0 * contract_basis(P, u);
    }
    const double Jqk = pick(k, Jq);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      double dcq[6];
      dC_F(b, q, dcq);
      double wq = 0.0, s = 0.0;
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        wq += b.wC[v] * dcq[v];
        s += t[v] * dcq[v];
      }
      D[hidx(q, 9 + k) * ds] = b.Jt * s + Jqk * wq;
    }
  }
  // F-F block and the F part of the gradient
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    double dcq[6];
    dC_F(b, q, dcq);
    double wq = 0.0;
#pragma unroll
    for (int v = 0; v < 6; ++v) wq += b.wC[v] * dcq[v];
    g[q] = b.Jt * wq;
    double WCq[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < 6; ++v) s += wCC[u][v] * dcq[v];
      WCq[u] = s;
    }
    const int i = q / 3, j = q % 3;
#pragma unroll
    for (int r = q; r < 9; ++r) {
      double dcr[6];
      dC_F(b, r, dcr);
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < 6; ++u) s += WCq[u] * dcr[u];
      const int k = r / 3, l = r % 3;
      if (i == k) s += 2.0 * GSG[3 * j + l];
      D[hidx(q, r) * ds] = b.Jt * s;
    }
  }
  // order-parameter gradient terms
  double We[NV + 1];
#pragma unroll
  for (int i = 0; i < NV + 1; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < NV + 1; ++j) t += cd.W[i][j] * eta[j];
    We[i] = t;
  }
  const double d0 = eta[0] - etan[0];
  const double n0 = neg_part(eta[0]);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    g[9 + k] += cd.dF0[k] + (We[k + 1] - We[0]) + cd.rho * ((eta[k + 1] - etan[k + 1]) - d0)
                + cd.eps * (neg_part(eta[k + 1]) - n0);
  }
}

}  // namespace mvpf
