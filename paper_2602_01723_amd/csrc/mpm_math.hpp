// Device math of the MLS-MPM substep: FP64 3x3 SVD / polar decomposition,
// the elastic Kirchhoff stresses and the plastic return maps.
//
// SVD: cyclic Jacobi on the symmetric matrix F^T F gives V and the squared
// singular values; the columns of F V are sorted by length and reduced by
// three Givens rotations (QR), which yields U in SO(3) and the singular
// values with the sign of det F carried by the last one (the convention of
// Irving et al. 2004 for inverted elements).  V in SO(3) as well.
//
// Stresses are Kirchhoff tau = P F^T (App. A.2 fixed corotated, StVK /
// Hencky and Neo-Hookean forms; App. B.1 Corotated, SigmaElasticity, StVK
// (Green-Lagrange), fluid and volume models).  Return maps follow App. A.2 /
// B.2 (identity, von Mises, Drucker-Prager with the Klar et al. 2016 plastic
// multiplier, fluid, sigma).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fmpm {

constexpr double kSigmaMin = 1e-4;  // log-strain floor for singular values
constexpr double kJMin = 1e-4;      // floor of J inside log J and 1/J
constexpr double kSigmaJLo = 0.05, kSigmaJHi = 1.2;  // sigma plasticity clamp of J

// model codes (the MPM_ELASTIC_* / MPM_PLASTIC_* values of the C ABI)
constexpr int kElasticFCR = 0, kElasticHencky = 1, kElasticNeoHookean = 2, kElasticStVK = 3, kElasticFluid = 4,
              kElasticVolume = 5;
constexpr int kPlasticNone = 0, kPlasticVonMises = 1, kPlasticDruckerPrager = 2, kPlasticFluid = 3,
              kPlasticSigma = 4;

struct Material {
  int32_t elastic;
  int32_t plastic;
  float yield_stress;
  float dp_alpha;  // sqrt(2/3) * 2 sin(phi) / (3 - sin(phi)), precomputed on the host
};

// -------------------------------------------------------------------------
// 3x3 helpers (row-major double[9])
// -------------------------------------------------------------------------
__device__ __forceinline__ double det3(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Reciprocal and reciprocal square root: the hardware estimates (relative
// error ~5e-8 on gfx950) refined by Newton steps; each step squares the error.
template <int STEPS>
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int k = 0; k < STEPS; ++k) r = r * fma(-x, r, 2.0);
  return r;
}
template <int STEPS>
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < STEPS; ++k) r = r * fma(-0.5 * x, r * r, 1.5);
  return r;
}

// One Jacobi rotation in plane (P, Q) of the symmetric S, accumulated into V.
// t = tan(phi) = 2 a_pq / (d + sign(d) sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp,
// the smaller of the two roots; c = 1 / sqrt(1 + t^2) with one Newton step on
// the hardware estimate, so c^2 + s^2 = 1 to about 1e-15.
template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(double S[3][3], double V[3][3]) {
  constexpr int R = 3 - P - Q;
  const double apq = S[P][Q];
  if (apq == 0.0) return;
  const double d = S[Q][Q] - S[P][P];
  const double h2 = fma(d, d, 4.0 * apq * apq);
  if (!(h2 > 1e-300)) return;
  const double h = h2 * rsq_nr<1>(h2);
  const double den = d + ((d < 0.0) ? -h : h);
  const double t = 2.0 * apq * rcp_nr<1>(den);
  const double c = rsq_nr<1>(fma(t, t, 1.0));
  const double s = t * c;
  const double arp = S[R][P], arq = S[R][Q];
  S[P][P] -= t * apq;
  S[Q][Q] += t * apq;
  S[P][Q] = 0.0;
  S[Q][P] = 0.0;
  const double nrp = c * arp - s * arq;
  const double nrq = s * arp + c * arq;
  S[R][P] = nrp;
  S[P][R] = nrp;
  S[R][Q] = nrq;
  S[Q][R] = nrq;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double vp = V[r][P], vq = V[r][Q];
    V[r][P] = c * vp - s * vq;
    V[r][Q] = s * vp + c * vq;
  }
}

template <int I, int J>
__device__ __forceinline__ void swap_cols_keep_det(double V[3][3], double lam[3]) {
  // exchange columns I and J and negate the new column J: det unchanged
  const double t = lam[I];
  lam[I] = lam[J];
  lam[J] = t;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double a = V[r][I];
    V[r][I] = V[r][J];
    V[r][J] = -a;
  }
}

// Givens rotation of rows (I, K) of B zeroing B[K][COL]; U <- U G^T.
template <int I, int K, int COL>
__device__ __forceinline__ void givens_qr(double B[3][3], double U[3][3]) {
  const double a = B[I][COL], b = B[K][COL];
  const double r2 = fma(a, a, b * b);
  if (r2 == 0.0) return;
  const double ir = rsq_nr<1>(r2);
  const double c = a * ir, s = b * ir;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double bi = B[I][j], bk = B[K][j];
    B[I][j] = c * bi + s * bk;
    B[K][j] = -s * bi + c * bk;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double ui = U[r][I], uk = U[r][K];
    U[r][I] = c * ui + s * uk;
    U[r][K] = -s * ui + c * uk;
  }
}

// F = U diag(sig) V^T, U, V in SO(3), |sig0| >= |sig1| >= |sig2|, sig0, sig1 >= 0.
// Jacobi on F^T F stops once its off-diagonal part E is below 1e-8 of the
// diagonal (sums of squares: 1e-16).  The QR of F V then has off-diagonal
// entries of about E / sig, which the factorisation drops: U diag(sig) V^T
// differs from F by about 1e-8 |F|, under the float32 rounding of the
// stored F (6e-8), while sig (the diagonal of R) is exact to second order.
__device__ __forceinline__ void svd3(const double* F, double U[3][3], double sig[3], double V[3][3]) {
  double S[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const double v = F[0 + i] * F[0 + j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
      S[i][j] = v;
      S[j][i] = v;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
    const double dia = S[0][0] * S[0][0] + S[1][1] * S[1][1] + S[2][2] * S[2][2];
    if (off <= 1e-16 * dia) break;
    jacobi_rotate<0, 1>(S, V);
    jacobi_rotate<0, 2>(S, V);
    jacobi_rotate<1, 2>(S, V);
  }
  double lam[3] = {S[0][0], S[1][1], S[2][2]};
  if (lam[0] < lam[1]) swap_cols_keep_det<0, 1>(V, lam);
  if (lam[0] < lam[2]) swap_cols_keep_det<0, 2>(V, lam);
  if (lam[1] < lam[2]) swap_cols_keep_det<1, 2>(V, lam);
  double B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[i][j] = F[3 * i + 0] * V[0][j] + F[3 * i + 1] * V[1][j] + F[3 * i + 2] * V[2][j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) U[i][j] = (i == j) ? 1.0 : 0.0;
  givens_qr<0, 1, 0>(B, U);
  givens_qr<0, 2, 0>(B, U);
  givens_qr<1, 2, 1>(B, U);
  sig[0] = B[0][0];
  sig[1] = B[1][1];
  sig[2] = B[2][2];
}

// A diag(d) B^T
__device__ __forceinline__ void diag_sandwich(const double A[3][3], const double* d, const double B[3][3],
                                              double* out) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) out[3 * i + j] = A[i][0] * d[0] * B[j][0] + A[i][1] * d[1] * B[j][1] + A[i][2] * d[2] * B[j][2];
}

// -------------------------------------------------------------------------
// Kirchhoff stresses (tau symmetric; full 3x3 returned)
// -------------------------------------------------------------------------

// Fixed corotated: tau = 2 mu (F - R) F^T + lam J (J - 1) I, R the polar rotation.
__device__ __forceinline__ void tau_fixed_corotated_R(const double* F, const double* R, double mu, double lam,
                                                      double* tau) {
  double P[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) P[k] = F[k] - R[k];
  const double J = det3(F);
  const double vol = lam * J * (J - 1.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double pf = P[3 * i + 0] * F[3 * j + 0] + P[3 * i + 1] * F[3 * j + 1] + P[3 * i + 2] * F[3 * j + 2];
      tau[3 * i + j] = 2.0 * mu * pf + ((i == j) ? vol : 0.0);
    }
}

// Rotation R of the polar decomposition F = R S by Newton's iteration
// X <- (X + X^-T) / 2 (Higham 1986), valid for det F > 0.  The iteration
// converges quadratically, so once an update is below 1e-8 the iterate is
// accurate to rounding.  Returns false if det X <= 0 or not converged; the
// caller then uses the SVD.
__device__ __forceinline__ bool polar_rotation_newton(const double* F, double* X) {
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = F[k];
  for (int it = 0; it < 16; ++it) {
    double cof[9];  // cofactor matrix = det(X) X^-T
    cof[0] = X[4] * X[8] - X[5] * X[7];
    cof[1] = X[5] * X[6] - X[3] * X[8];
    cof[2] = X[3] * X[7] - X[4] * X[6];
    cof[3] = X[2] * X[7] - X[1] * X[8];
    cof[4] = X[0] * X[8] - X[2] * X[6];
    cof[5] = X[1] * X[6] - X[0] * X[7];
    cof[6] = X[1] * X[5] - X[2] * X[4];
    cof[7] = X[2] * X[3] - X[0] * X[5];
    cof[8] = X[0] * X[4] - X[1] * X[3];
    const double det = X[0] * cof[0] + X[1] * cof[1] + X[2] * cof[2];
    if (!(det > 0.0)) return false;
    const double hd = 0.5 * rcp_nr<2>(det);
    double diff = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double y = fma(0.5, X[k], hd * cof[k]);
      const double dk = y - X[k];
      diff = fma(dk, dk, diff);
      X[k] = y;
    }
    if (diff < 1e-16) return true;
  }
  return false;
}

// Hencky (logarithmic strain): tau = U diag(2 mu eps + lam tr(eps)) U^T,
// from the principal log strains eps.
__device__ __forceinline__ void tau_hencky_eps(const double U[3][3], const double* e, double mu, double lam,
                                               double* tau) {
  double d[3];
  const double tr = e[0] + e[1] + e[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) d[k] = 2.0 * mu * e[k] + lam * tr;
  diag_sandwich(U, d, U, tau);
}

// Elastic models in closed form of F (no SVD):
//   Neo-Hookean  tau = mu (F F^T - I) + lam log(J+) I
//   StVK         tau = F (2 mu E + lam tr(E) I) F^T, E = (F^T F - I) / 2
//   fluid        tau = lam J (J - 1) I
//   volume       tau = kappa (J - 1 / J+) I, kappa = 2/3 mu + lam
// with J+ = max(J, 1e-4).
__device__ __forceinline__ void tau_closed_form(int model, const double* F, double mu, double lam, double* tau) {
  const double J = det3(F);
  if (model == kElasticNeoHookean) {
    const double p = lam * log(fmax(J, kJMin));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double b = F[3 * i] * F[3 * j] + F[3 * i + 1] * F[3 * j + 1] + F[3 * i + 2] * F[3 * j + 2];
        tau[3 * i + j] = mu * (b - (i == j ? 1.0 : 0.0)) + (i == j ? p : 0.0);
      }
    return;
  }
  if (model == kElasticStVK) {
    double S[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        S[3 * i + j] = 0.5 * (F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j] - (i == j ? 1.0 : 0.0));
    const double tr = S[0] + S[4] + S[8];
#pragma unroll
    for (int k = 0; k < 9; ++k) S[k] = 2.0 * mu * S[k] + (k % 4 == 0 ? lam * tr : 0.0);
    double FS[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        FS[3 * i + j] = F[3 * i] * S[j] + F[3 * i + 1] * S[3 + j] + F[3 * i + 2] * S[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        tau[3 * i + j] = FS[3 * i] * F[3 * j] + FS[3 * i + 1] * F[3 * j + 1] + FS[3 * i + 2] * F[3 * j + 2];
    return;
  }
  const double p = (model == kElasticFluid) ? lam * J * (J - 1.0)
                                            : (2.0 / 3.0 * mu + lam) * (J - 1.0 / fmax(J, kJMin));
#pragma unroll
  for (int k = 0; k < 9; ++k) tau[k] = (k % 4 == 0) ? p : 0.0;
}

// -------------------------------------------------------------------------
// Return maps.  Input: F_trial (FP64) and its SVD.  Output: F' and the
// principal log strains of F' (U, V unchanged), which the Hencky stress of
// the next substep uses directly.
// -------------------------------------------------------------------------
__device__ __forceinline__ void return_map(const Material& mat, double mu, double lam, const double* Ftr,
                                           const double U[3][3], const double* sig, const double V[3][3],
                                           double* Fout, double* eps_out) {
#pragma unroll
  for (int k = 0; k < 9; ++k) Fout[k] = Ftr[k];
  double e[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    e[k] = log(fmax(sig[k], kSigmaMin));
    eps_out[k] = e[k];
  }
  if (mat.plastic == 0) return;
  const double tr = e[0] + e[1] + e[2];
  const double mean = tr * (1.0 / 3.0);
  const double eh[3] = {e[0] - mean, e[1] - mean, e[2] - mean};
  const double nrm = sqrt(eh[0] * eh[0] + eh[1] * eh[1] + eh[2] * eh[2]);
  double dgamma;
  if (mat.plastic == 1) {  // von Mises
    dgamma = nrm - (double)mat.yield_stress / (2.0 * mu);
  } else {  // Drucker-Prager
    if (tr > 0.0) {
      const double one[3] = {1.0, 1.0, 1.0};
      diag_sandwich(U, one, V, Fout);
      eps_out[0] = eps_out[1] = eps_out[2] = 0.0;
      return;
    }
    dgamma = nrm + (3.0 * lam + 2.0 * mu) / (2.0 * mu) * tr * (double)mat.dp_alpha;
  }
  if (!(dgamma > 0.0)) return;
  const double scale = dgamma / nrm;
  double s2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    eps_out[k] = e[k] - scale * eh[k];
    s2[k] = exp(eps_out[k]);
  }
  diag_sandwich(U, s2, V, Fout);
}

// Deformation update and stress of one particle.  Ftr is the trial
// deformation gradient (FP64).  Computes the plastic return map (when the
// material has one) into Fout and the Kirchhoff stress tau of Fout for the
// particle's elastic model.  One SVD at most: the closed-form models need
// one only under von Mises / Drucker-Prager; fluid and sigma plasticity use
// det F alone; a fixed-corotated particle takes its rotation from Newton's
// polar iteration, falling back to the SVD for inverted or degenerate F.
// apply_plasticity = false evaluates the stress of Ftr as given.
__device__ __forceinline__ void update_and_stress(const Material& mat, double mu, double lam, const double* Ftr,
                                                  bool apply_plasticity, bool want_stress, double* Fout,
                                                  double* tau) {
  const bool svd_plastic =
      apply_plasticity && (mat.plastic == kPlasticVonMises || mat.plastic == kPlasticDruckerPrager);
  const bool j_plastic = apply_plasticity && (mat.plastic == kPlasticFluid || mat.plastic == kPlasticSigma);
  // Fs: the trial F, or its volumetric projection cbrt(J) I (fluid / sigma
  // plasticity), whose stress the elastic model then gives
  double Fs[9];
  if (j_plastic) {
    double J = det3(Ftr);
    if (mat.plastic == kPlasticSigma) J = fmin(fmax(J, kSigmaJLo), kSigmaJHi);
    const double c = cbrt(J);
#pragma unroll
    for (int k = 0; k < 9; ++k) Fs[k] = (k % 4 == 0) ? c : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Fs[k] = Ftr[k];
  }
  // one SVD call site for every model (the code is inlined per call site):
  // von Mises / Drucker-Prager, Hencky, and the fixed-corotated fallback
  const bool closed = mat.elastic >= kElasticNeoHookean;
  double R[9];
  bool have_R = false;
  if (!closed && !svd_plastic && mat.elastic == kElasticFCR) {
    if (!want_stress) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Fout[k] = Fs[k];
      return;
    }
    have_R = polar_rotation_newton(Fs, R);
  }
  double U[3][3], V[3][3], eps[3];
  if (svd_plastic || (!closed && !have_R)) {
    double sig[3];
    svd3(Fs, U, sig, V);
    if (svd_plastic) {
      return_map(mat, mu, lam, Fs, U, sig, V, Fout, eps);
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) Fout[k] = Fs[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) eps[k] = log(fmax(sig[k], kSigmaMin));
    }
    if (!closed && mat.elastic == kElasticFCR) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) R[3 * i + j] = U[i][0] * V[j][0] + U[i][1] * V[j][1] + U[i][2] * V[j][2];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Fout[k] = Fs[k];
  }
  if (!want_stress) return;
  if (closed)
    tau_closed_form(mat.elastic, Fout, mu, lam, tau);
  else if (mat.elastic == kElasticFCR)
    tau_fixed_corotated_R(Fout, R, mu, lam, tau);
  else
    tau_hencky_eps(U, eps, mu, lam, tau);
}

}  // namespace fmpm
