// Reverse-mode (adjoint) kernels of the MLS-MPM substep: the stresses of the
// fixed-corotated, Hencky, Neo-Hookean, StVK, fluid and volume models and
// the von Mises, Drucker-Prager, fluid and sigma return maps
// (included once, by fastmpm.hip after mpm_kernels.hpp).
//
// Forward substep k on state s_k = (x, v, C, F), per particle p and node i:
//   tau_p = 2 mu (F - R) F^T + lam J (J - 1) I            (App. B.1, Corotated)
//   A_p   = m_p C_p - D dt V_p tau_p,  D = 4 / dx^2
//   m_i   = sum_p w_ip m_p,  mv_i = sum_p w_ip (m_p v_p + A_p (x_i - x_p))
//   vh_i  = mv_i / m_i + dt g   (active nodes; 0 on walls and empty nodes)
//   v'_p  = sum_i w_ip vh_i,  C'_p = D sum_i w_ip vh_i (x_i - x_p)^T
//   x'_p  = x_p + dt v'_p,    F'_p = (I + dt C'_p) F_p
// with w_ip the quadratic B-spline weights of x_p.
//
// Reverse, given the adjoints (xb', vb', Cb', Fb') of s_{k+1}:
//   k_adj_g2p  (particle-parallel, scatter):  Fb = (I + dt C')^T Fb',
//     Cbt = Cb' + dt Fb' F^T, vbt = vb' + dt xb', xb = xb';
//     vhb_i += w (vbt + D Cbt dpos)  (global FP32 atomics);
//     xb += [vh_i . vbt + D vh_i^T Cbt dpos] grad_x w - D w Cbt^T vh_i
//   k_adj_p2g  (particle-parallel, gather):  per node
//     mvb_i = vhb_i / m_i, mb_i = -vhb_i . (mv_i / m_i) / m_i  (active nodes),
//     wb = mb_i m_p + mvb_i . (m_p v_p + A_p dpos),  vb += m_p w mvb_i,
//     Ab += w mvb_i dpos^T,  xb += wb grad_x w - w A_p^T mvb_i;
//   then Cb = m_p Ab, taub = -D dt V_p Ab, and the stress adjoint (FP64)
//     Fb += 2 mu (taub F + taub^T (F - R) - R [c]x) + lam (2J - 1) J tr(taub) F^-T,
//     c = (tr(S) I - S)^-1 axial(R^T M - M^T R), M = taub F, S = R^T F,
//     mub = <taub, 2 (F - R) F^T>, lamb = J (J - 1) tr(taub),
//   and the parameter gradients
//     g_logE += mub mu + lamb lam,
//     g_nu   += -mub mu / (1 + nu) + lamb E (1 + 2 nu^2) / ((1 + nu)(1 - 2 nu))^2.
#pragma once

#include <type_traits>

#include "mpm_kernels.hpp"

namespace fmpm {

struct AdjArgs {
  // state s_k of the substep being reversed (internal order, plane stride N)
  const float* x;
  const float* v;
  const float* C;
  const float* F;
  const float4* prm;   // mass, vol0, mu, lam
  const float* lnE;    // log E (internal order)
  const float* nu;     // Poisson ratio (internal order)
  int64_t N;
  const int* chunk_start;  // per-scene chunks of kBlock particles
  const int* chunk_batch;
  const float4* grid;  // (mv, m) of substep k
  float4* vhb;         // adjoint of the grid velocity (xyz), zeroed before k_adj_g2p
  // adjoint state: in = adjoint of s_{k+1}, out = adjoint of s_k
  float* ax;
  float* av;
  float* aC;
  float* aF;
  float* g_lnE;        // accumulated parameter gradients (internal order)
  float* g_nu;
  const int* mat;      // material id (internal order)
  const Material* mats;
  int n_materials;
  int n;
  int bound;
  float dt;
  float g[3];
  // deterministic mode (k_adj_g2p<true>): per-scene bound of the
  // grid-velocity adjoint contributions (float bits, both slots of the
  // scene), the per-item bounds k_adj_bound stores, the scenes' range
  // factors and the 64-bit fixed-point grid
  unsigned* fxb;
  float2* fxi;
  const double* fxk;
  unsigned long long* gfx;
  unsigned* gflag;  // flags of gfx's 4^3-node blocks the scatter adds into (k_fx_grid_blocks)
};

__device__ __forceinline__ void bspline_dw(float f, float* dw) {
  dw[0] = f - 1.5f;          // d/df 0.5 (1.5 - f)^2
  dw[1] = -2.0f * (f - 1.0f);  // d/df 0.75 - (f - 1)^2
  dw[2] = f - 0.5f;          // d/df 0.5 (f - 0.5)^2
}

__device__ __forceinline__ bool grid_active(float m, int ix, int iy, int iz, int n, int bd) {
  const bool wall = ix < bd || iy < bd || iz < bd || ix >= n - bd || iy >= n - bd || iz >= n - bd;
  return (m > 0.0f) && !wall;
}

// (mv / m, 1 / m) of a node whose velocity the grid update computes (m > 0,
// off the walls); zero for every other node
__device__ __forceinline__ float4 node_vim(float4 g, int ix, int iy, int iz, int n, int bd) {
  if (!grid_active(g.w, ix, iy, iz, n, bd)) return make_float4(0.f, 0.f, 0.f, 0.f);
  const float im = 1.0f / g.w;
  return make_float4(g.x * im, g.y * im, g.z * im, im);
}

// Polar rotation of F (det F > 0 expected), SVD fallback.
__device__ __forceinline__ void polar_rotation(const double* F, double* R) {
  if (polar_rotation_newton(F, R)) return;
  double U[3][3], V[3][3], sg[3];
  svd3(F, U, sg, V);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) R[3 * i + j] = U[i][0] * V[j][0] + U[i][1] * V[j][1] + U[i][2] * V[j][2];
}

// Adjoint of the fixed-corotated Kirchhoff stress: Fb += dL/dF, mub, lamb.
__device__ __forceinline__ void tau_fcr_adjoint(const double* F, const double* R, double mu, double lam,
                                                const double* tb, double* Fb, double& mub, double& lamb) {
  const double J = det3(F);
  double trtb = tb[0] + tb[4] + tb[8];
  // mub = <tb, 2 (F - R) F^T>
  double P[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) P[k] = F[k] - R[k];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      s += tb[3 * i + j] * (P[3 * i] * F[3 * j] + P[3 * i + 1] * F[3 * j + 1] + P[3 * i + 2] * F[3 * j + 2]);
  mub = 2.0 * s;
  lamb = J * (J - 1.0) * trtb;
  // M = tb F, S = R^T F
  double M[9], S[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      M[3 * i + j] = tb[3 * i] * F[j] + tb[3 * i + 1] * F[3 + j] + tb[3 * i + 2] * F[6 + j];
      S[3 * i + j] = R[i] * F[j] + R[3 + i] * F[3 + j] + R[6 + i] * F[6 + j];
    }
  // Y = R^T M; a = axial(Y - Y^T)
  double Y[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Y[3 * i + j] = R[i] * M[j] + R[3 + i] * M[3 + j] + R[6 + i] * M[6 + j];
  const double av[3] = {Y[7] - Y[5], Y[2] - Y[6], Y[3] - Y[1]};
  // K = tr(S) I - S (symmetrised), c = K^-1 a
  const double trS = S[0] + S[4] + S[8];
  double K[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) K[3 * i + j] = ((i == j) ? trS : 0.0) - 0.5 * (S[3 * i + j] + S[3 * j + i]);
  double cof[9];
  cof[0] = K[4] * K[8] - K[5] * K[7];
  cof[1] = K[5] * K[6] - K[3] * K[8];
  cof[2] = K[3] * K[7] - K[4] * K[6];
  cof[3] = K[2] * K[7] - K[1] * K[8];
  cof[4] = K[0] * K[8] - K[2] * K[6];
  cof[5] = K[1] * K[6] - K[0] * K[7];
  cof[6] = K[1] * K[5] - K[2] * K[4];
  cof[7] = K[2] * K[3] - K[0] * K[5];
  cof[8] = K[0] * K[4] - K[1] * K[3];
  const double detK = K[0] * cof[0] + K[1] * cof[1] + K[2] * cof[2];
  const double idet = (detK != 0.0) ? 1.0 / detK : 0.0;
  // K^-1 = cof^T / det (K symmetric, so cof symmetric as well)
  double c[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) c[i] = (cof[i] * av[0] + cof[3 + i] * av[1] + cof[6 + i] * av[2]) * idet;
  // [c]x and R [c]x
  const double cx[9] = {0.0, -c[2], c[1], c[2], 0.0, -c[0], -c[1], c[0], 0.0};
  // F^-T = cof(F) / J
  double cf[9];
  cf[0] = F[4] * F[8] - F[5] * F[7];
  cf[1] = F[5] * F[6] - F[3] * F[8];
  cf[2] = F[3] * F[7] - F[4] * F[6];
  cf[3] = F[2] * F[7] - F[1] * F[8];
  cf[4] = F[0] * F[8] - F[2] * F[6];
  cf[5] = F[1] * F[6] - F[0] * F[7];
  cf[6] = F[1] * F[5] - F[2] * F[4];
  cf[7] = F[2] * F[3] - F[0] * F[5];
  cf[8] = F[0] * F[4] - F[1] * F[3];
  // J F^-T = cof(F); term lam (2J - 1) tr(tb) J F^-T
  const double kv = lam * (2.0 * J - 1.0) * trtb;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double tbF = M[3 * i + j];
      const double tbtP = tb[i] * P[j] + tb[3 + i] * P[3 + j] + tb[6 + i] * P[6 + j];  // (tb^T P)_ij
      const double Rc = R[3 * i] * cx[j] + R[3 * i + 1] * cx[3 + j] + R[3 * i + 2] * cx[6 + j];
      Fb[3 * i + j] += 2.0 * mu * (tbF + tbtP - Rc) + kv * cf[3 * i + j];
    }
}

// Adjoint of the closed-form models (Fb += dL/dF, mub, lamb), with
// cof = J F^-T = dJ/dF and tb the cotangent of tau:
//   Neo-Hookean  Fb += mu (tb + tb^T) F + lam tr(tb) F^-T [J > 1e-4]
//   StVK         Fb += (tb + tb^T) F S + F sym(Eb), Sb = F^T tb F,
//                Eb = 2 mu Sb + lam tr(Sb) I, mub = 2 <Sb, E>, lamb = tr(Sb) tr(E)
//   fluid        Fb += lam tr(tb) (2J - 1) cof
//   volume       Fb += kappa tr(tb) (1 + [J > 1e-4] / J^2) cof, kappab = tr(tb) (J - 1/J+)
__device__ __forceinline__ void tau_closed_form_adjoint(int model, const double* F, double mu, double lam,
                                                        const double* tb, double* Fb, double& mub, double& lamb) {
  const double J = det3(F);
  const double trtb = tb[0] + tb[4] + tb[8];
  double cof[9];
  cof[0] = F[4] * F[8] - F[5] * F[7];
  cof[1] = F[5] * F[6] - F[3] * F[8];
  cof[2] = F[3] * F[7] - F[4] * F[6];
  cof[3] = F[2] * F[7] - F[1] * F[8];
  cof[4] = F[0] * F[8] - F[2] * F[6];
  cof[5] = F[1] * F[6] - F[0] * F[7];
  cof[6] = F[1] * F[5] - F[2] * F[4];
  cof[7] = F[2] * F[3] - F[0] * F[5];
  cof[8] = F[0] * F[4] - F[1] * F[3];
  if (model == kElasticNeoHookean) {
    const double kj = (J > kJMin) ? lam * trtb / J : 0.0;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double b = F[3 * i] * F[3 * j] + F[3 * i + 1] * F[3 * j + 1] + F[3 * i + 2] * F[3 * j + 2];
        s += tb[3 * i + j] * (b - (i == j ? 1.0 : 0.0));
        // (tb + tb^T) F
        Fb[3 * i + j] += mu * ((tb[3 * i] + tb[i]) * F[j] + (tb[3 * i + 1] + tb[3 + i]) * F[3 + j] +
                               (tb[3 * i + 2] + tb[6 + i]) * F[6 + j]) +
                         kj * cof[3 * i + j];
      }
    mub += s;
    lamb += trtb * log(fmax(J, kJMin));
    return;
  }
  if (model == kElasticStVK) {
    double E[9], S[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        E[3 * i + j] = 0.5 * (F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j] - (i == j ? 1.0 : 0.0));
    const double trE = E[0] + E[4] + E[8];
#pragma unroll
    for (int k = 0; k < 9; ++k) S[k] = 2.0 * mu * E[k] + (k % 4 == 0 ? lam * trE : 0.0);
    double T[9], FS[9], TF[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) T[k] = tb[k] + tb[3 * (k % 3) + k / 3];  // tb + tb^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        FS[3 * i + j] = F[3 * i] * S[j] + F[3 * i + 1] * S[3 + j] + F[3 * i + 2] * S[6 + j];
        TF[3 * i + j] = tb[3 * i] * F[j] + tb[3 * i + 1] * F[3 + j] + tb[3 * i + 2] * F[6 + j];  // tb F
      }
    // Sb = F^T tb F
    double Sb[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Sb[3 * i + j] = F[i] * TF[j] + F[3 + i] * TF[3 + j] + F[6 + i] * TF[6 + j];
    const double trSb = Sb[0] + Sb[4] + Sb[8];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) s += Sb[k] * E[k];
    mub += 2.0 * s;
    lamb += trSb * trE;
    double Es[9];  // sym(Eb), Eb = 2 mu Sb + lam tr(Sb) I
#pragma unroll
    for (int k = 0; k < 9; ++k)
      Es[k] = mu * (Sb[k] + Sb[3 * (k % 3) + k / 3]) + (k % 4 == 0 ? lam * trSb : 0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Fb[3 * i + j] += T[3 * i] * FS[j] + T[3 * i + 1] * FS[3 + j] + T[3 * i + 2] * FS[6 + j] +
                         F[3 * i] * Es[j] + F[3 * i + 1] * Es[3 + j] + F[3 * i + 2] * Es[6 + j];
    return;
  }
  double dp;  // d(pressure)/dJ times tr(tb)
  if (model == kElasticFluid) {
    dp = lam * trtb * (2.0 * J - 1.0);
    lamb += trtb * J * (J - 1.0);
  } else {
    const double kappa = 2.0 / 3.0 * mu + lam;
    dp = kappa * trtb * (1.0 + ((J > kJMin) ? 1.0 / (J * J) : 0.0));
    const double kb = trtb * (J - 1.0 / fmax(J, kJMin));
    mub += 2.0 / 3.0 * kb;
    lamb += kb;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Fb[k] += dp * cof[k];
}

// Adjoint of the Hencky stress tau = mu L + (lam/2) tr(L) I, L = log(F F^T)
// = 2 U diag(eps) U^T:  with G = mu sym(taub) + (lam/2) tr(taub) I and the
// divided differences D_ij of log at lambda = sigma^2 (D_ii = 1/lambda_i),
//   bb = U (D o (U^T G U)) U^T,  Fb += 2 bb F,
//   mub = <taub, 2 U diag(eps) U^T>,  lamb = tr(taub) sum(eps).
__device__ __forceinline__ void tau_hencky_adjoint(const double* F, const double U[3][3], const double* sig,
                                                   double mu, double lam, const double* tb, double* Fb, double& mub,
                                                   double& lamb) {
  double e[3], l[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    e[k] = log(fmax(sig[k], kSigmaMin));
    l[k] = sig[k] * sig[k];
  }
  const double trtb = tb[0] + tb[4] + tb[8];
  // mub = <taub, 2 U diag(e) U^T>
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s += tb[3 * i + j] * (U[i][0] * e[0] * U[j][0] + U[i][1] * e[1] * U[j][1] + U[i][2] * e[2] * U[j][2]);
  mub = 2.0 * s;
  lamb = trtb * (e[0] + e[1] + e[2]);
  // G in the eigenbasis: H = U^T G U
  double G[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) G[3 * i + j] = mu * 0.5 * (tb[3 * i + j] + tb[3 * j + i]) + ((i == j) ? 0.5 * lam * trtb : 0.0);
  double H[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double h = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) h += U[a][i] * G[3 * a + b] * U[b][j];
      H[3 * i + j] = h;
    }
  // D o H
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double d;
      if (i == j) {
        d = 1.0 / l[i];
      } else {
        const double dl = l[i] - l[j];
        d = (fabs(dl) > 1e-6 * fmax(l[i], l[j])) ? 2.0 * (e[i] - e[j]) / dl : 2.0 / (l[i] + l[j]);
      }
      H[3 * i + j] *= d;
    }
  // bb = U H U^T, Fb += 2 bb F
  double bb[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t += U[i][a] * H[3 * a + b] * U[j][b];
      bb[3 * i + j] = t;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Fb[3 * i + j] += 2.0 * (bb[3 * i] * F[j] + bb[3 * i + 1] * F[3 + j] + bb[3 * i + 2] * F[6 + j]);
}

// Adjoint of the plastic return map F' = Z(F_trial) (App. A.2, App. B.2):
// Fbo is the cotangent of F', Fb receives that of F_trial, and the adjoints
// of mu and lam are added to mub, lamb.
//  * fluid, sigma: F' = cbrt(J) I, so Fb = tr(Fbo) cof(F) / (3 cbrt(J)^2)
//    (zero where sigma plasticity clamps J).
//  * von Mises, Drucker-Prager: with F = U diag(s) V^T, eps = log s,
//    m = mean(eps), n = eps_hat / |eps_hat|, a flow step is
//    F' = U diag(g) V^T, g_k = exp(m + r n_k), r = yield / (2 mu) (von Mises)
//    or r = -3 beta m, beta = (3 lam + 2 mu) / (2 mu) alpha (Drucker-Prager);
//    the Drucker-Prager tension case is g = 1.  For a function of this form,
//    with G = U^T Fbo V:
//      Pb_ii = s_i^-1 sum_k G_kk g_k d eps'_k / d eps_i,
//      Pb_ij = (a + b)/2 G_ij + (a - b)/2 G_ji  (i != j),
//      a = (g_i - g_j) / (s_i - s_j),  b = (g_i + g_j) / (s_i + s_j),
//    and Fb = U Pb V^T.  a is taken as g_j / s_j * expm1(c L) / expm1(L),
//    L = eps_i - eps_j, c = r / |eps_hat| (g_i = K s_i^c), which stays exact
//    as s_i -> s_j.  Singular values under the log floor do not move eps.
__device__ __forceinline__ void return_map_adjoint(const Material& mat, double mu, double lam, const double* F,
                                                   const double* Fbo, double* Fb, double& mub, double& lamb) {
  if (mat.plastic == kPlasticFluid || mat.plastic == kPlasticSigma) {
    const double J = det3(F);
    if (mat.plastic == kPlasticSigma && (J < kSigmaJLo || J > kSigmaJHi)) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Fb[k] = 0.0;
      return;
    }
    const double c = cbrt(J);
    const double kf = (Fbo[0] + Fbo[4] + Fbo[8]) / (3.0 * c * c);
    Fb[0] = kf * (F[4] * F[8] - F[5] * F[7]);
    Fb[1] = kf * (F[5] * F[6] - F[3] * F[8]);
    Fb[2] = kf * (F[3] * F[7] - F[4] * F[6]);
    Fb[3] = kf * (F[2] * F[7] - F[1] * F[8]);
    Fb[4] = kf * (F[0] * F[8] - F[2] * F[6]);
    Fb[5] = kf * (F[1] * F[6] - F[0] * F[7]);
    Fb[6] = kf * (F[1] * F[5] - F[2] * F[4]);
    Fb[7] = kf * (F[2] * F[3] - F[0] * F[5]);
    Fb[8] = kf * (F[0] * F[4] - F[1] * F[3]);
    return;
  }
  if (mat.plastic != kPlasticVonMises && mat.plastic != kPlasticDruckerPrager) {
#pragma unroll
    for (int k = 0; k < 9; ++k) Fb[k] = Fbo[k];
    return;
  }
  double U[3][3], V[3][3], sg[3], e[3];
  svd3(F, U, sg, V);
#pragma unroll
  for (int k = 0; k < 3; ++k) e[k] = log(fmax(sg[k], kSigmaMin));
  const double tr = e[0] + e[1] + e[2];
  const double m = tr * (1.0 / 3.0);
  const double eh[3] = {e[0] - m, e[1] - m, e[2] - m};
  const double nrm = sqrt(eh[0] * eh[0] + eh[1] * eh[1] + eh[2] * eh[2]);
  // the branch the forward return map took
  bool tension = false;
  double r = 0.0, drde = 0.0, beta = 0.0;
  if (mat.plastic == kPlasticVonMises) {
    r = (double)mat.yield_stress / (2.0 * mu);
    if (!(nrm - r > 0.0)) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Fb[k] = Fbo[k];
      return;
    }
  } else if (tr > 0.0) {
    tension = true;
  } else {
    beta = (3.0 * lam + 2.0 * mu) / (2.0 * mu) * (double)mat.dp_alpha;
    if (!(nrm + beta * tr > 0.0)) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Fb[k] = Fbo[k];
      return;
    }
    r = -beta * tr;
    drde = -beta;
  }
  // G = U^T Fbo V
  double G[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t += U[a][i] * Fbo[3 * a + b] * V[b][j];
      G[i][j] = t;
    }
  double g[3] = {1.0, 1.0, 1.0}, P[3][3];
  const double cc = tension ? 0.0 : r / nrm;
  if (tension) {
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i][i] = 0.0;
  } else {
    double n[3], h[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      n[k] = eh[k] / nrm;
      g[k] = exp(m + r * n[k]);
      h[k] = G[k][k] * g[k];
    }
    const double H = h[0] + h[1] + h[2];
    const double nh = n[0] * h[0] + n[1] * h[1] + n[2] * h[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double d = H * (1.0 / 3.0) + cc * (h[i] - H * (1.0 / 3.0) - n[i] * nh) + drde * nh;
      P[i][i] = (sg[i] > kSigmaMin) ? d / sg[i] : 0.0;
    }
    // r-bar = n . h
    if (mat.plastic == kPlasticVonMises) {
      mub += -nh * r / mu;
    } else {
      const double bb = -tr * nh;  // beta-bar
      const double al = (double)mat.dp_alpha;
      lamb += bb * 1.5 * al / mu;
      mub += -bb * 1.5 * al * lam / (mu * mu);
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i + 1; j < 3; ++j) {
      double a = 0.0;
      if (!tension) {
        if (sg[i] > kSigmaMin && sg[j] > kSigmaMin) {
          const double L = e[i] - e[j];
          const double ratio = (fabs(L) < 1e-6) ? cc * (1.0 + 0.5 * (cc - 1.0) * L) : expm1(cc * L) / expm1(L);
          a = g[j] / sg[j] * ratio;
        } else if (sg[i] != sg[j]) {
          a = (g[i] - g[j]) / (sg[i] - sg[j]);
        }
      }
      double den = sg[i] + sg[j];
      if (fabs(den) < 1e-12) den = (den < 0.0) ? -1e-12 : 1e-12;
      const double b = (g[i] + g[j]) / den;
      const double gij = G[i][j], gji = G[j][i];
      P[i][j] = 0.5 * (a + b) * gij + 0.5 * (a - b) * gji;
      P[j][i] = 0.5 * (a + b) * gji + 0.5 * (a - b) * gij;
    }
  // Fb = U P V^T
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t += U[i][a] * P[a][b] * V[j][b];
      Fb[3 * i + j] = t;
    }
}

// Reverse of one substep's return map, particle-parallel: on entry aF holds
// the adjoint of F_{k+1}, on exit that of F_trial = (I + dt C') F_k, formed
// from F_k and C' = C_{k+1} of the recomputed states the way the forward
// pass formed it; the adjoints of mu and lam go into the parameter
// gradients.  Particles without a return map, and particles the forward
// pass skipped, keep aF.
__global__ __launch_bounds__(256) void k_adj_return_map(const float* x, const float* F, const float* Cn, const float4* prm, const int* mat,
                                 const Material* mats, int n_materials, const float* lnE, const float* nu, float dt,
                                 int n, float* aF, float* g_lnE, float* g_nu, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int mid = mat[i];
  mid = (mid >= 0 && mid < n_materials) ? mid : 0;
  const Material mt = mats[mid];
  if (mt.plastic == kPlasticNone) return;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int b;
    float f;
    ok &= cell_of(x[k * N + i], n, b, f);
  }
  if (!ok) return;
  double Fd[9], Cp[9], Fbo[9], Ftr[9], Fb[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Fd[k] = (double)F[k * N + i];
    Cp[k] = (double)Cn[k * N + i];
    Fbo[k] = (double)aF[k * N + i];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double acc = Fd[3 * r + c];
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += (double)dt * Cp[3 * r + k] * Fd[3 * k + c];
      Ftr[3 * r + c] = acc;
    }
  const float4 pm = prm[i];
  const double mu = (double)pm.z, lam = (double)pm.w;
  double mub = 0.0, lamb = 0.0;
  return_map_adjoint(mt, mu, lam, Ftr, Fbo, Fb, mub, lamb);
#pragma unroll
  for (int k = 0; k < 9; ++k) aF[k * N + i] = (float)Fb[k];
  if (mub != 0.0 || lamb != 0.0) {
    const double E = exp((double)lnE[i]);
    const double nv = (double)nu[i];
    const double den = (1.0 + nv) * (1.0 - 2.0 * nv);
    g_lnE[i] += (float)(mub * mu + lamb * lam);
    g_nu[i] += (float)(-mub * mu / (1.0 + nv) + lamb * E * (1.0 + 2.0 * nv * nv) / (den * den));
  }
}

// --------------------------------------------------------------------------
// Reverse of G2P (and of the x, F updates).  Same work items as the forward
// substep kernel: per item the node velocities of the stencil box are read
// into an LDS tile (grid update folded in) and the velocity adjoint
// accumulates in an LDS f64 tile (staggered node order), flushed with one
// global FP32 atomic per node and channel.  Items whose box exceeds the
// tile use global memory.
// --------------------------------------------------------------------------
struct AdjItems {
  const int* item_start;  // [n_items + 1]
  const int* item_batch;
  const int* n_items;
  int* counter;           // zero at launch
  int tile_cap;
  const int* box_in;      // per-item base-cell boxes of the state (NULL: a pass over x)
};

// Deterministic mode: each item's bound of |w (vbt + D Cbt dpos)| over its
// particles and their 27 nodes (w <= 0.75^3, |dpos| <= 1.5 dx per axis),
// stored in both channels of a.fxi[item] (k_fx_fold then forms each
// scene's bound).  One workgroup per item.
__global__ __launch_bounds__(256) void k_adj_bound(AdjArgs a, AdjItems it) {
  __shared__ float wmax[4];
  const int item = blockIdx.x;
  if (item >= *it.n_items) return;
  const int64_t N = a.N;
  const float dx = 1.0f / (float)a.n, D = 4.0f * (float)a.n * (float)a.n;
  float mx = 0.0f;  // this lane's largest bound
  for (int i = it.item_start[item] + (int)threadIdx.x; i < it.item_start[item + 1]; i += blockDim.x) {
    int b[3];
    float f[3];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) ok &= cell_of(a.x[k * N + i], a.n, b[k], f[k]);
    if (!ok) continue;
    float bnd = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      float row = 0.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float t = a.aC[(3 * r + c) * N + i];
#pragma unroll
        for (int k = 0; k < 3; ++k) t += a.dt * a.aF[(3 * r + k) * N + i] * a.F[(3 * c + k) * N + i];
        row += fabsf(t);
      }
      bnd = fmaxf(bnd, fabsf(a.av[r * N + i] + a.dt * a.ax[r * N + i]) + D * 1.5f * dx * row);
    }
    bnd *= 0.421875f;
    if (bnd <= 3.0e38f) mx = fmaxf(mx, bnd);  // NaN and overflow stay out of the scale
  }
  mx = wave_maxf(mx);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmaxf(mx, wmax[w]);
    a.fxi[item] = make_float2(mx, mx);
  }
}

// Three workgroups per CU (48 KB of LDS each; at most 168 VGPRs) in the
// default mode, where the host launches 1.5 times the forward's workgroup
// count; two in deterministic mode (its fixed-point scatter would spill).
template <bool DET = false>
__global__ __launch_bounds__(kBlock, DET ? 2 : 3) void k_adj_g2p(AdjArgs a, AdjItems it) {
  __shared__ double ptile[3 * kTileCapMax];
  // deterministic mode: the same LDS as 64-bit fixed point at the scene's scale
  unsigned long long* const pu = reinterpret_cast<unsigned long long*>(ptile);
  __shared__ float gtile[3 * kTileCapMax];
  __shared__ int red[8 * (kBlock / 64)];
  __shared__ int item_s;
  const int n = a.n;
  const int64_t N = a.N;
  const float inv_dx = (float)n, dx = 1.0f / (float)n, D = 4.0f * inv_dx * inv_dx;
  const int n_items = *it.n_items;
  SubstepArgs ga{};
  ga.n = n;
  ga.bound = a.bound;
  ga.dt = a.dt;
  ga.g[0] = a.g[0];
  ga.g[1] = a.g[1];
  ga.g[2] = a.g[2];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_s = atomicAdd(it.counter, 1);
    __syncthreads();
    const int item = item_s;
    if (item >= n_items) break;
    const int start = it.item_start[item], end = it.item_start[item + 1];
    const int64_t gbase = (int64_t)it.item_batch[item] * n * n * n;
    double s_fx = 1.0;
    if (DET) {
      const int scene = it.item_batch[item];
      s_fx = fx_scale(fx_range(a.fxb, a.fxk, scene) * (double)__uint_as_float(a.fxb[4 * scene]));
    }
    int box[6];
    if (it.box_in) {
#pragma unroll
      for (int k = 0; k < 6; ++k) box[k] = it.box_in[6 * item + k];
    } else {
      int lo[3] = {0x3fffffff, 0x3fffffff, 0x3fffffff}, hi[3] = {-0x3fffffff, -0x3fffffff, -0x3fffffff};
      for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        int b[3];
        float f[3];
        bool in = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) in &= cell_of(a.x[k * N + i], n, b[k], f[k]);
        if (in) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            lo[k] = min(lo[k], b[k]);
            hi[k] = max(hi[k], b[k]);
          }
        }
      }
      block_minmax(lo, hi, red, box);
    }
    const bool empty = box[0] > box[3];
    const int gx = box[3] - box[0] + 3, gy = box[4] - box[1] + 3, gz = box[5] - box[2] + 3;
    // x stride padded like the forward P2G tile (the scatter's LDS banks)
    const int sz = gy * gz + kPadX;
    const int GT = empty ? 0 : (gx - 1) * sz + (gy - 1) * gz + gz;
    const bool lds = !empty && GT <= it.tile_cap;
    if (lds) {
      for (int t = threadIdx.x; t < GT; t += kBlock) {
        const int ti = t / sz, tr = t - ti * sz;
        const int tj = min(tr / gz, gy - 1), tk = tr - (tr / gz) * gz;  // padding entries load a valid node
        const int ix = box[0] + ti, iy = box[1] + tj, iz = box[2] + tk;
        float vv[3];
        grid_velocity(a.grid[gbase + ((int64_t)ix * n + iy) * n + iz], ix, iy, iz, ga, vv);
        gtile[t] = vv[0];
        gtile[kTileCapMax + t] = vv[1];
        gtile[2 * kTileCapMax + t] = vv[2];
        ptile[t] = 0.0;
        ptile[kTileCapMax + t] = 0.0;
        ptile[2 * kTileCapMax + t] = 0.0;
      }
    }
    __syncthreads();
    for (int sub = start; sub < end; sub += kBlock) {
      const int i = sub + (int)threadIdx.x;
      if (i >= end) break;
      float xp[3], Fp[9], xb[3], vb[3], Cb[9], Fbo[9];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xp[k] = a.x[k * N + i];
        xb[k] = a.ax[k * N + i];
        vb[k] = a.av[k * N + i];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        Fp[k] = a.F[k * N + i];
        Cb[k] = a.aC[k * N + i];
        Fbo[k] = a.aF[k * N + i];
      }
      int b[3];
      float f[3];
      bool ok = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) ok &= cell_of(xp[k], n, b[k], f[k]);
      if (!ok) continue;  // skipped in the forward pass: the adjoint passes through
      float w[3][3], dw[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        bspline_w(f[k], w[k]);
        bspline_dw(f[k], dw[k]);
      }
      const int a0 = (b[0] - box[0]) * sz + (b[1] - box[1]) * gz + (b[2] - box[2]);
      // C' of the forward pass from the stencil's node velocities
      auto node_v = [&](int ox, int oy, int oz, float* out) {
        if (lds) {
          const int t = a0 + ox * sz + oy * gz + oz;
          out[0] = gtile[t];
          out[1] = gtile[kTileCapMax + t];
          out[2] = gtile[2 * kTileCapMax + t];
        } else {
          const int ix = b[0] + ox, iy = b[1] + oy, iz = b[2] + oz;
          grid_velocity(a.grid[gbase + ((int64_t)ix * n + iy) * n + iz], ix, iy, iz, ga, out);
        }
      };
      // B = sum w v (o - f)^T dx = dx (M - v f^T); the tile path sums axis
      // by axis, the global-memory fallback node by node in a rolled loop
      float vs[3], M[3][3], B[3][3];
      if (lds) {
        auto tile_v = [&](int ox, int oy, int oz, float* out) {
          const int t = a0 + ox * sz + oy * gz + oz;
          out[0] = gtile[t];
          out[1] = gtile[kTileCapMax + t];
          out[2] = gtile[2 * kTileCapMax + t];
        };
        g2p_moments(w[0], w[1], w[2], tile_v, vs, M);
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) vs[c] = M[c][0] = M[c][1] = M[c][2] = 0.f;
#pragma unroll 1
        for (int o = 0; o < 27; ++o) {
          const int ox = o / 9, oy = (o / 3) % 3, oz = o % 3;
          float vi[3];
          node_v(ox, oy, oz, vi);
          const float wt = sel3(w[0], ox) * sel3(w[1], oy) * sel3(w[2], oz);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float wv = wt * vi[c];
            vs[c] += wv;
            M[c][0] += (float)ox * wv;
            M[c][1] += (float)oy * wv;
            M[c][2] += (float)oz * wv;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) B[r][c] = dx * (M[r][c] - vs[r] * f[c]);
      float Fb[9], Cbt[9], vbt[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          float s = Fbo[3 * r + c];
#pragma unroll
          for (int k = 0; k < 3; ++k) s += a.dt * D * B[k][r] * Fbo[3 * k + c];
          Fb[3 * r + c] = s;
          float t = Cb[3 * r + c];
#pragma unroll
          for (int k = 0; k < 3; ++k) t += a.dt * Fbo[3 * r + k] * Fp[3 * c + k];
          Cbt[3 * r + c] = t;
        }
#pragma unroll
      for (int k = 0; k < 3; ++k) vbt[k] = vb[k] + a.dt * xb[k];
      // staggered node order (lanes of one cell hit different nodes): lane
      // group g visits offset (k + g_axis) mod 3 at step k on each axis.  x
      // and y loops stay rolled (register use); the z values sit in
      // compile-time indexed tables
      const int g = (threadIdx.x & 63) % 27;
      const int gs[3] = {g / 9, (g / 3) % 3, g % 3};
      int roz[3];
      float wrz[3], dwrz[3], dprz[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        roz[k] = rot3(gs[2], k);
        wrz[k] = sel3(w[2], roz[k]);
        dwrz[k] = inv_dx * sel3(dw[2], roz[k]);
        dprz[k] = ((float)roz[k] - f[2]) * dx;
      }
      float xo[3] = {xb[0], xb[1], xb[2]};
      // one loop nest for the tile and one for global memory (the choice is
      // uniform per item), so the node loops carry no per-node test
      auto scatter = [&](auto tile_c) {
        constexpr bool TILE = decltype(tile_c)::value;
#pragma unroll 1
      for (int kx = 0; kx < 3; ++kx) {
        // x-axis values by selection (a rolled loop keeps register use down)
        const int ox = rot3(gs[0], kx);
        const float wx = sel3(w[0], ox), dwx = inv_dx * sel3(dw[0], ox), dpx = ((float)ox - f[0]) * dx;
#pragma unroll 1
        for (int ky = 0; ky < 3; ++ky) {
          const int oy = rot3(gs[1], ky);
          const float wy = sel3(w[1], oy), dwy = inv_dx * sel3(dw[1], oy), dpy = ((float)oy - f[1]) * dx;
#pragma unroll
          for (int kz = 0; kz < 3; ++kz) {
            const int oz = roz[kz];
            float vho[3];
            if (TILE) {
              const int t = a0 + ox * sz + oy * gz + oz;
              vho[0] = gtile[t];
              vho[1] = gtile[kTileCapMax + t];
              vho[2] = gtile[2 * kTileCapMax + t];
            } else {
              node_v(ox, oy, oz, vho);
            }
            const float wz = wrz[kz];
            const float wt = wx * wy * wz;
            const float gw[3] = {dwx * wy * wz, wx * dwy * wz, wx * wy * dwrz[kz]};
            const float dp[3] = {dpx, dpy, dprz[kz]};
            float cd[3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
              cd[r] = Cbt[3 * r] * dp[0] + Cbt[3 * r + 1] * dp[1] + Cbt[3 * r + 2] * dp[2];
            float wb = 0.f, gv[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
              const float gval = vbt[r] + D * cd[r];
              gv[r] = wt * gval;
              wb += vho[r] * gval;
            }
            if (TILE) {
              const int t = a0 + ox * sz + oy * gz + oz;
              if (DET) {
#pragma unroll
                for (int r = 0; r < 3; ++r) atomicAdd(&pu[r * kTileCapMax + t], fx_bits(gv[r], s_fx));
              } else {
#pragma unroll
                for (int r = 0; r < 3; ++r) atomicAdd(&ptile[r * kTileCapMax + t], (double)gv[r]);
              }
            } else {
              const int ix = b[0] + ox, iy = b[1] + oy, iz = b[2] + oz;
              const int64_t node = gbase + ((int64_t)ix * n + iy) * n + iz;
              if (DET) {
                const int nbn = (n + 3) >> 2;
                a.gflag[(int64_t)it.item_batch[item] * nbn * nbn * nbn + ((int64_t)(ix >> 2) * nbn + (iy >> 2)) * nbn +
                        (iz >> 2)] = 1u;
#pragma unroll
                for (int r = 0; r < 3; ++r)
                  atomicAdd(a.gfx + 4 * node + r, (unsigned long long)fx_value(fx_bits(gv[r], s_fx)));
              } else {
                float* gp = (float*)&a.vhb[node];
#pragma unroll
                for (int r = 0; r < 3; ++r) atomicAdd(gp + r, gv[r]);
              }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float ctv = Cbt[c] * vho[0] + Cbt[3 + c] * vho[1] + Cbt[6 + c] * vho[2];
              xo[c] += wb * gw[c] - D * wt * ctv;
            }
          }
        }
      }
      };
      if (lds)
        scatter(std::true_type{});
      else
        scatter(std::false_type{});
#pragma unroll
      for (int k = 0; k < 3; ++k) a.ax[k * N + i] = xo[k];
#pragma unroll
      for (int k = 0; k < 9; ++k) a.aF[k * N + i] = Fb[k];
    }
    if (lds) {
      __syncthreads();
      if (DET) {  // flag the 4^3-node blocks the tile covers (nodes box.lo .. box.hi + 2)
        const int nbn = (n + 3) >> 2;
        const int bx0 = box[0] >> 2, by0 = box[1] >> 2, bz0 = box[2] >> 2;
        const int nx = ((box[3] + 2) >> 2) - bx0 + 1, ny = ((box[4] + 2) >> 2) - by0 + 1,
                  nz = ((box[5] + 2) >> 2) - bz0 + 1;
        const int64_t sbase = (int64_t)it.item_batch[item] * nbn * nbn * nbn;
        for (int t = threadIdx.x; t < nx * ny * nz; t += kBlock) {
          const int bx = bx0 + t / (ny * nz), by = by0 + (t / nz) % ny, bz = bz0 + t % nz;
          a.gflag[sbase + ((int64_t)bx * nbn + by) * nbn + bz] = 1u;
        }
      }
      for (int t = threadIdx.x; t < GT; t += kBlock) {
        const int ti = t / sz, tr = t - ti * sz;
        const int tj = tr / gz, tk = tr - tj * gz;
        if (tj >= gy) continue;  // padding
        const int64_t node = gbase + ((int64_t)(box[0] + ti) * n + (box[1] + tj)) * n + (box[2] + tk);
        if (DET) {  // integer sums at the scene's scale: exact, in any order
          const long long q0 = fx_value(pu[t]), q1 = fx_value(pu[kTileCapMax + t]),
                          q2 = fx_value(pu[2 * kTileCapMax + t]);
          if (q0 == 0 && q1 == 0 && q2 == 0) continue;
          atomicAdd(a.gfx + 4 * node + 0, (unsigned long long)q0);
          atomicAdd(a.gfx + 4 * node + 1, (unsigned long long)q1);
          atomicAdd(a.gfx + 4 * node + 2, (unsigned long long)q2);
        } else {
          const double v0 = ptile[t], v1 = ptile[kTileCapMax + t], v2 = ptile[2 * kTileCapMax + t];
          if (v0 == 0.0 && v1 == 0.0 && v2 == 0.0) continue;
          float* gp = (float*)&a.vhb[node];
          atomicAdd(gp + 0, (float)v0);
          atomicAdd(gp + 1, (float)v1);
          atomicAdd(gp + 2, (float)v2);
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// Reverse of the grid update and of P2G, stress and Lame parameters
// --------------------------------------------------------------------------
// One particle of the P2G / stress reverse; tile(ix, iy, iz, gv, gb) and
// glob(...) fetch the node's node_vim (mv / m, 1 / m) and grid-velocity
// adjoint from the LDS tile (lds set) or from global memory.
template <typename TileFn, typename GlobFn>
__device__ __forceinline__ void adj_p2g_particle(const AdjArgs& a, int i, bool lds, TileFn tile, GlobFn glob) {
  const int n = a.n;
  const int64_t N = a.N;
  const float inv_dx = (float)n, dx = 1.0f / (float)n, D = 4.0f * inv_dx * inv_dx;
  float xp[3], vp[3], Cp[9], xb[3];
  double Fd[9], Fb[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xp[k] = a.x[k * N + i];
    vp[k] = a.v[k * N + i];
    xb[k] = a.ax[k * N + i];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Cp[k] = a.C[k * N + i];
    Fd[k] = (double)a.F[k * N + i];
    Fb[k] = (double)a.aF[k * N + i];
  }
  const float4 prm = a.prm[i];
  const float mass = prm.x;
  const double mu = (double)prm.z, lam = (double)prm.w;
  int b[3];
  float f[3];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) ok &= cell_of(xp[k], n, b[k], f[k]);
  if (!ok) return;  // skipped in the forward pass: the adjoint passes through
  float vb[3] = {0.f, 0.f, 0.f}, Cb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  {
    int mid = a.mat[i];
    mid = (mid >= 0 && mid < a.n_materials) ? mid : 0;
    const int el = a.mats[mid].elastic;
    const bool fcr = el == kElasticFCR;
    double R[9], tau[9], U[3][3], V[3][3], sg[3];
    if (fcr) {
      polar_rotation(Fd, R);
      tau_fixed_corotated_R(Fd, R, mu, lam, tau);
    } else if (el >= kElasticNeoHookean) {
      tau_closed_form(el, Fd, mu, lam, tau);
    } else {
      svd3(Fd, U, sg, V);
      double e[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) e[k] = log(fmax(sg[k], kSigmaMin));
      tau_hencky_eps(U, e, mu, lam, tau);
    }
    const float ks = D * a.dt * prm.y;
    float A[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = mass * Cp[k] - ks * (float)tau[k];
    // Per node o (weight w_o, weight gradient gw_o, adjoints mvb_o, mb_o of
    // its mv, m): the forward added w_o (m v + A (o - f) dx) to mv_o and
    // w_o m to m_o.  With g = m v - A f dx the momentum term is g + A o dx,
    // and the sums over o that do not involve gw reduce to
    //   S0 = sum w mvb,  M1[r][c] = sum w mvb_r o_c:
    //   vb = m S0,  Ab = dx (M1 - S0 f^T),  xb -= A^T S0.
    // The remaining term xb += sum_o wb_o gw_o, wb_o = m mb_o + mvb_o . (g + A o dx),
    // is summed node by node.
    float w[3][3], dwi[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float dw[3];
      bspline_w(f[k], w[k]);
      bspline_dw(f[k], dw);
#pragma unroll
      for (int o = 0; o < 3; ++o) dwi[k][o] = inv_dx * dw[o];
    }
    float g[3], Ad[9];  // Ad = A dx (A itself is not kept: register use)
#pragma unroll
    for (int k = 0; k < 9; ++k) Ad[k] = A[k] * dx;
#pragma unroll
    for (int r = 0; r < 3; ++r) g[r] = mass * vp[r] - (Ad[3 * r] * f[0] + Ad[3 * r + 1] * f[1] + Ad[3 * r + 2] * f[2]);
    float S0[3] = {0.f, 0.f, 0.f};
    float M1[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    // one stencil node; ox, oy, oz are compile-time constants on the tile
    // path and the selections fold away
    auto visit = [&](int ox, int oy, int oz, const float4& gv, const float4& gb) {
      const float im = gv.w;
      if (!(im > 0.0f)) return;  // no mass, or a wall node: its velocity does not depend on mv, m
      const float mvb[3] = {gb.x * im, gb.y * im, gb.z * im};
      const float mb = -(gb.x * gv.x + gb.y * gv.y + gb.z * gv.z) * im;  // -(gb . mv) / m^2
      float wb = mass * mb;
#pragma unroll
      for (int r = 0; r < 3; ++r)
        wb += mvb[r] * (((g[r] + Ad[3 * r] * (float)ox) + Ad[3 * r + 1] * (float)oy) + Ad[3 * r + 2] * (float)oz);
      const float wx = sel3(w[0], ox), wy = sel3(w[1], oy), wz = sel3(w[2], oz);
      const float wxy = wx * wy, wyz = wy * wz;
      const float gw[3] = {sel3(dwi[0], ox) * wyz, wx * sel3(dwi[1], oy) * wz, wxy * sel3(dwi[2], oz)};
#pragma unroll
      for (int c = 0; c < 3; ++c) xb[c] += wb * gw[c];
      const float wt = wxy * wz;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const float wm = wt * mvb[r];
        S0[r] += wm;
        if (ox) M1[r][0] += (float)ox * wm;
        if (oy) M1[r][1] += (float)oy * wm;
        if (oz) M1[r][2] += (float)oz * wm;
      }
    };
    // one branch per particle: the tile path is unrolled, the global-memory
    // fallback (items whose box exceeds the tile) stays a rolled loop so the
    // rare path does not multiply the code
    if (lds) {
#pragma unroll
      for (int ox = 0; ox < 3; ++ox)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            float4 gv, gb;
            tile(b[0] + ox, b[1] + oy, b[2] + oz, gv, gb);
            visit(ox, oy, oz, gv, gb);
          }
    } else {
#pragma unroll 1
      for (int o = 0; o < 27; ++o) {
        const int ox = o / 9, oy = (o / 3) % 3, oz = o % 3;
        float4 gv, gb;
        glob(b[0] + ox, b[1] + oy, b[2] + oz, gv, gb);
        visit(ox, oy, oz, gv, gb);
      }
    }
    float Ab[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      vb[r] = mass * S0[r];
#pragma unroll
      for (int c = 0; c < 3; ++c) Ab[3 * r + c] = dx * (M1[r][c] - f[c] * S0[r]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) xb[c] -= inv_dx * (Ad[c] * S0[0] + Ad[3 + c] * S0[1] + Ad[6 + c] * S0[2]);
    // A = m C - ks tau
#pragma unroll
    for (int k = 0; k < 9; ++k) Cb[k] = mass * Ab[k];
    double tb[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) tb[k] = -(double)ks * (double)Ab[k];
    double mub = 0.0, lamb = 0.0;
    if (fcr)
      tau_fcr_adjoint(Fd, R, mu, lam, tb, Fb, mub, lamb);
    else if (el >= kElasticNeoHookean)
      tau_closed_form_adjoint(el, Fd, mu, lam, tb, Fb, mub, lamb);
    else
      tau_hencky_adjoint(Fd, U, sg, mu, lam, tb, Fb, mub, lamb);
    const double E = exp((double)a.lnE[i]);
    const double nv = (double)a.nu[i];
    const double den = (1.0 + nv) * (1.0 - 2.0 * nv);
    a.g_lnE[i] += (float)(mub * mu + lamb * lam);
    a.g_nu[i] += (float)(-mub * mu / (1.0 + nv) + lamb * E * (1.0 + 2.0 * nv * nv) / (den * den));
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.ax[k * N + i] = xb[k];
    a.av[k * N + i] = vb[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    a.aC[k * N + i] = Cb[k];
    a.aF[k * N + i] = (float)Fb[k];
  }
}

// Persistent over the work items of the last sort: each item's box of grid
// nodes ((mv, m) and the grid-velocity adjoint) is staged in LDS, the
// particles then gather from it (global memory when the box exceeds the tile).
__global__ __launch_bounds__(kBlock, 2) void k_adj_p2g(AdjArgs a, AdjItems it) {
  __shared__ float4 gm_t[kTileCapMax];  // node_vim of the item's node box
  __shared__ float4 gb_t[kTileCapMax];
  __shared__ int red[8 * (kBlock / 64)];
  __shared__ int item_s;
  const int n = a.n;
  const int64_t N = a.N;
  const int n_items = *it.n_items;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_s = atomicAdd(it.counter, 1);
    __syncthreads();
    const int item = item_s;
    if (item >= n_items) break;
    const int start = it.item_start[item], end = it.item_start[item + 1];
    const int64_t gbase = (int64_t)it.item_batch[item] * n * n * n;
    int box[6];
    if (it.box_in) {
#pragma unroll
      for (int k = 0; k < 6; ++k) box[k] = it.box_in[6 * item + k];
    } else {
      int lo[3] = {0x3fffffff, 0x3fffffff, 0x3fffffff}, hi[3] = {-0x3fffffff, -0x3fffffff, -0x3fffffff};
      for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        int b[3];
        float f[3];
        bool in = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) in &= cell_of(a.x[k * N + i], n, b[k], f[k]);
        if (in) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            lo[k] = min(lo[k], b[k]);
            hi[k] = max(hi[k], b[k]);
          }
        }
      }
      block_minmax(lo, hi, red, box);
    }
    const bool empty = box[0] > box[3];
    const int gx = box[3] - box[0] + 3, gy = box[4] - box[1] + 3, gz = box[5] - box[2] + 3;
    const int GT = empty ? 0 : gx * gy * gz;
    const bool lds = !empty && GT <= it.tile_cap;
    if (lds) {
      for (int t = threadIdx.x; t < GT; t += kBlock) {
        const int tk = t % gz, tq = t / gz;
        const int tj = tq % gy, ti = tq / gy;
        const int64_t node = gbase + ((int64_t)(box[0] + ti) * n + (box[1] + tj)) * n + (box[2] + tk);
        gm_t[t] = node_vim(a.grid[node], box[0] + ti, box[1] + tj, box[2] + tk, n, a.bound);
        gb_t[t] = a.vhb[node];
      }
    }
    __syncthreads();
    auto tile = [&](int ix, int iy, int iz, float4& gm, float4& gb) {
      const int t = ((ix - box[0]) * gy + (iy - box[1])) * gz + (iz - box[2]);
      gm = gm_t[t];
      gb = gb_t[t];
    };
    auto glob = [&](int ix, int iy, int iz, float4& gm, float4& gb) {
      const int64_t node = gbase + ((int64_t)ix * n + iy) * n + iz;
      gm = node_vim(a.grid[node], ix, iy, iz, n, a.bound);
      gb = a.vhb[node];
    };
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) adj_p2g_particle(a, i, lds, tile, glob);
  }
}

// a[j] += b[j], c[j] += d[j]
__global__ void k_add2(float* a, const float* b, float* c, const float* d, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  a[j] += b[j];
  c[j] += d[j];
}

// cotangent of L = sum_p w_p |x_p - x*_p|^2: g_x = 2 w_p (x_p - x*_p)
__global__ void k_position_loss_grad(const float* x, const float* xt, const float* w, float* gx, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const float s = 2.0f * w[j];
#pragma unroll
  for (int c = 0; c < 3; ++c) gx[c * N + j] = s * (x[c * N + j] - xt[c * N + j]);
}

// plain copy of `count` floats
__global__ void k_copy_f32(float* out, const float* in, int64_t count) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) out[j] = in[j];
}

}  // namespace fmpm
