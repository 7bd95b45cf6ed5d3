// Local (quadrature-point) derivatives of the penalised incremental potential
// density with respect to q = (F_00..F_22 row-major, eta_1..eta_6).
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

namespace mvpf {

// Material card on the device, in the sample frame.
struct DevCard {
  double dU[6][6];     // U_k - I (k = 1..6) as symmetric components
  double L0[6][6];     // austenite stiffness, Voigt (engineering shear strain)
  double dL[6][6][6];  // L_k - L_0
  double dF0[6];       // F_k - F_0
  double W[7][7];      // double-obstacle coefficients, zero diagonal
  double Sw[6][6];     // condensed Hessian of 1/2 eta^T W eta w.r.t. eta_hat
  double Mg[6][6];     // gradient-energy species matrix: psi_g = 1/2 Mg_kl grad eta_k . grad eta_l
  double rho;
  double eps;
  int pade;
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

__host__ __device__ constexpr int hidx(int p, int q) {  // packed upper triangle, p <= q < 15
  return p * 15 - (p * (p - 1)) / 2 + (q - p);
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
  double wEta[6]; // partial dw/deta_k at fixed C
  double dh[6][6];  // engineering components of dH_v
  double h[6];      // engineering H
  double T[6];      // L H (tensor components)
  double Binv[9];
  double H[9];
};

// Hencky energy (Pade order PD) and its first C-derivatives.
template <int PD>
__device__ __forceinline__ void local_base(const double F[9], const double eh[6], const DevCard& cd,
                                           LocalBase& b) {
  using P = Pade<PD>;
  double Ft[6];
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    double s = (v < 3) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) s += eh[k] * cd.dU[k][v];
    Ft[v] = s;
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
      for (int k = 0; k < 6; ++k) s += eh[k] * cd.dL[k][i][j];
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
  for (int k = 0; k < 6; ++k) {
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

// Symmetric components of dC along variable q (0..8: F_ij row-major; 9..14: eta).
__device__ __forceinline__ void dC_of(const LocalBase& b, const DevCard& cd, int q, double dc[6],
                                      double dcf[9]) {
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
    full_from_sym(cd.dU[k], dU);
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

// a[i] for a runtime i in 0..5 from six values (selection, no indexing)
__device__ __forceinline__ double pick6(int i, double a0, double a1, double a2, double a3, double a4, double a5) {
  double r = a0;
  r = (i == 1) ? a1 : r;
  r = (i == 2) ? a2 : r;
  r = (i == 3) ? a3 : r;
  r = (i == 4) ? a4 : r;
  r = (i == 5) ? a5 : r;
  return r;
}

// Q_k = G dU_k (full)
__device__ __forceinline__ void Q_of(const LocalBase& b, const DevCard& cd, int k, double Q[9]) {
  double dU[9];
  full_from_sym(cd.dU[k], dU);
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

// Gradient of the local density: g[15].
template <int PD>
__device__ __forceinline__ void local_gradient(const double F[9], const double eh[6], const double ehn[6],
                                               const DevCard& cd, double g[15]) {
  LocalBase b;
  local_base<PD>(F, eh, cd, b);
#pragma unroll
  for (int q = 0; q < 15; ++q) {
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
      full_from_sym(cd.dU[k], dU);
      mm(b.G, dU, Q);
      const double trQ = Q[0] + Q[4] + Q[8];
      g[q] = b.Jt * (wq + b.wEta[k]) + b.Jt * trQ * b.w;
    }
  }
  // order-parameter terms: chemical, double obstacle, viscous, penalty
  double eta[7], etan[7];
  double s = 0.0, sn = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) { eta[k + 1] = eh[k]; etan[k + 1] = ehn[k]; s += eh[k]; sn += ehn[k]; }
  eta[0] = 1.0 - s;
  etan[0] = 1.0 - sn;
  double We[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < 7; ++j) t += cd.W[i][j] * eta[j];
    We[i] = t;
  }
  const double d0 = eta[0] - etan[0];
  const double n0 = neg_part(eta[0]);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    g[9 + k] += cd.dF0[k] + (We[k + 1] - We[0]) + cd.rho * ((eta[k + 1] - etan[k + 1]) - d0)
                + cd.eps * (neg_part(eta[k + 1]) - n0);
  }
}

// Gradient and packed upper-triangular Hessian of the local density; entry
// hidx(p, q) of the Hessian is stored to D[hidx(p, q) * ds] as soon as it is
// known (nothing of it is kept in registers).
template <int PD>
__device__ __forceinline__ void local_hessian(const double F[9], const double eh[6], const double ehn[6],
                                              const DevCard& cd, double g[15], double* __restrict__ D,
                                              int64_t ds) {
  using P = Pade<PD>;
  LocalBase b;
  local_base<PD>(F, eh, cd, b);
  // ---- second derivatives in C-space -------------------------------------
  double wCC[6][6];
  double wCeta[6][6];  // [v][k]
  {
    double Lm[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double s = cd.L0[i][j];
#pragma unroll
        for (int k = 0; k < 6; ++k) s += eh[k] * cd.dL[k][i][j];
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
    for (int k = 0; k < 6; ++k) {
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
  double dce[6][6], wqe[6], Jq[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
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
  double eta[7], etan[7];
  {
    double s = 0.0, sn = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) { eta[k + 1] = eh[k]; etan[k + 1] = ehn[k]; s += eh[k]; sn += ehn[k]; }
    eta[0] = 1.0 - s;
    etan[0] = 1.0 - sn;
  }
  const double pen0 = (eta[0] < 0.0) ? cd.eps : 0.0;
  // Runtime (not unrolled) loops over the pairs k <= l: unrolled, the
  // compiler keeps every Q_l product of all pairs live at once.  Values of
  // the per-eta register arrays are picked by static-index selection.
#pragma unroll 1
  for (int k = 0; k < 6; ++k) {
    double Qk[9], SQ[9], Rk[9], Uk[9], WCk[6], dk[6], wek[6];
    Q_of(b, cd, k, Qk);
    mm(Sf, Qk, SQ);
    mm(b.C, SQ, Rk);  // C S Q_k
    mm(SQ, b.C, Uk);  // S Q_k C
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      dk[v] = pick6(k, dce[0][v], dce[1][v], dce[2][v], dce[3][v], dce[4][v], dce[5][v]);
      wek[v] = pick6(k, wCeta[v][0], wCeta[v][1], wCeta[v][2], wCeta[v][3], wCeta[v][4], wCeta[v][5]);
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < 6; ++v) s += wCC[u][v] * dk[v];
      WCk[u] = s;
    }
    const double trk = Qk[0] + Qk[4] + Qk[8];
    const double Jqk = pick6(k, Jq[0], Jq[1], Jq[2], Jq[3], Jq[4], Jq[5]);
    const double wqk = pick6(k, wqe[0], wqe[1], wqe[2], wqe[3], wqe[4], wqe[5]);
    const double etak = pick6(k, eta[1], eta[2], eta[3], eta[4], eta[5], eta[6]);
#pragma unroll 1
    for (int l = k; l < 6; ++l) {
      double Ql[9], SQl[9], Rl[9], dl[6], wel[6];
      Q_of(b, cd, l, Ql);
      mm(Sf, Ql, SQl);
      mm(b.C, SQl, Rl);  // C S Q_l
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        dl[v] = pick6(l, dce[0][v], dce[1][v], dce[2][v], dce[3][v], dce[4][v], dce[5][v]);
        wel[v] = pick6(l, wCeta[v][0], wCeta[v][1], wCeta[v][2], wCeta[v][3], wCeta[v][4], wCeta[v][5]);
      }
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < 6; ++u) s += WCk[u] * dl[u];
      s += 2.0 * (trprod(Rk, Ql) + trprod(Rl, Qk) + ddot9(Uk, Ql));
#pragma unroll
      for (int v = 0; v < 6; ++v) s += wel[v] * dk[v] + wek[v] * dl[v];
      const double trl = Ql[0] + Ql[4] + Ql[8];
      const double Jkl = b.Jt * (trk * trl - trprod(Qk, Ql));
      const double Jql = pick6(l, Jq[0], Jq[1], Jq[2], Jq[3], Jq[4], Jq[5]);
      const double wql = pick6(l, wqe[0], wqe[1], wqe[2], wqe[3], wqe[4], wqe[5]);
      double val = b.Jt * s + Jqk * wql + Jql * wqk + Jkl * b.w;
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
  for (int k = 0; k < 6; ++k) {
    double Q[9], P[9], t[6];
    Q_of(b, cd, k, Q);
    mm(Sf, Q, P);  // S G dU_k
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      double wdk = 0.0;
#pragma unroll
      for (int v = 0; v < 6; ++v)
        wdk += wCC[u][v] * pick6(k, dce[0][v], dce[1][v], dce[2][v], dce[3][v], dce[4][v], dce[5][v]);
      t[u] = wdk + pick6(k, wCeta[u][0], wCeta[u][1], wCeta[u][2], wCeta[u][3], wCeta[u][4], wCeta[u][5]) -
             2.0 * contract_basis(P, u);
    }
    const double Jqk = pick6(k, Jq[0], Jq[1], Jq[2], Jq[3], Jq[4], Jq[5]);
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
  double We[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < 7; ++j) t += cd.W[i][j] * eta[j];
    We[i] = t;
  }
  const double d0 = eta[0] - etan[0];
  const double n0 = neg_part(eta[0]);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    g[9 + k] += cd.dF0[k] + (We[k + 1] - We[0]) + cd.rho * ((eta[k + 1] - etan[k + 1]) - d0)
                + cd.eps * (neg_part(eta[k + 1]) - n0);
  }
}

}  // namespace mvpf
