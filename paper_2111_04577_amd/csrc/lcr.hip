// Log-conformation polymer update (Sec. 2.2, eqs. NS17-NS24; Sec. 3.2.3, eqs. NS40-NS46).
//
// Theta = log c is advanced by the two-stage TVD Runge-Kutta scheme of eqs. NS42 and NS44 with
// u^{n+1} fixed; each stage diagonalises its own Theta (eqs. NS43, NS45) and forms
//   RH = -div(u Theta) + (Omega Theta - Theta Omega) + 2 B
//        - (1/Wi) e^{-Theta} [I + alpha (e^Theta - I)] (e^Theta - I)          (eq. NS41)
// in the eigenframe, where M = R^T K R (K_ij = du_i/dx_j, eq. NS23), B = R diag(m_ii) R^T and
// the commutator has entries omega_ij (theta_j - theta_i) (eq. NS24). That product is formed as
// (e^d m_ij + m_ji) d / expm1(d), d = theta_j - theta_i, equal to the paper's expression for
// distinct eigenvalues and to its limit m_ij + m_ji for equal ones (at c = I the paper's rule
// Omega = 0, B = sym K); the relaxation sign is the one that relaxes c to I. The second stage
// also diagonalises Theta^{n+1} (a Jacobi started in the eigenframe of Theta^(1), O(dt) away)
// and writes tau_p = (1 - beta)/Wi (c - I) (eq. NS46), formed as V diag(expm1(theta)) V^T.
//
// One thread per coarse cell. The per-cell eigensolve (cyclic Jacobi) and the source are FP64
// in both precision forms; the advection is the stress form's flux form (central, or WENO-Z
// face values) with zero wall flux.
#include "coarse.hpp"
#include "weno.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;

// Cyclic Jacobi for a symmetric 3x3 matrix: on exit a is diagonal (the eigenvalues) and the
// columns of v are the eigenvectors. Stops when the off-diagonal mass is below 1e-32 of the
// diagonal mass (relative 1e-16 per entry, FP64 round-off) or after 16 sweeps.
__device__ __forceinline__ void jacobi3(double a[3][3], double v[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off == 0.0 || off <= 1e-32 * dia) break;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int p = r == 2 ? 1 : 0, q = r == 0 ? 1 : 2;
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      // rotation that annihilates a[p][q] (the smaller of the two angles)
      const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      // a <- J^T a J with J the (p, q) rotation
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double akp = a[k][p], akq = a[k][q];
        a[k][p] = c * akp - s * akq;
        a[k][q] = s * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double apk = a[p][k], aqk = a[q][k];
        a[p][k] = c * apk - s * aqk;
        a[q][k] = s * apk + c * aqk;
      }
      a[p][q] = a[q][p] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double vkp = v[k][p], vkq = v[k][q];
        v[k][p] = c * vkp - s * vkq;
        v[k][q] = s * vkp + c * vkq;
      }
    }
  }
}

// omega_ij (theta_j - theta_i) of eq. NS24 for d = theta_j - theta_i, without overflow:
// (e^d m_ij + m_ji) d / expm1(d) for d < 0, (m_ij + e^{-d} m_ji) d / -expm1(-d) for d > 0.
__device__ __forceinline__ double commutator_entry(double d, double mij, double mji) {
  if (d == 0.0) return mij + mji;
  if (d < 0.0) return (exp(d) * mij + mji) * (d / expm1(d));
  return (mij + exp(-d) * mji) * (d / -expm1(-d));
}

// symmetric 3x3 <-> six components (xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ void unpack6(const double t[6], double m[3][3]) {
  m[0][0] = t[0];
  m[1][1] = t[1];
  m[2][2] = t[2];
  m[0][1] = m[1][0] = t[3];
  m[0][2] = m[2][0] = t[4];
  m[1][2] = m[2][1] = t[5];
}

// R diag(d) R^T as six components
__device__ __forceinline__ void rdr6(const double R[3][3], const double d[3], double out[6]) {
  const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int a = pa[m], b = pb[m];
    out[m] = R[a][0] * d[0] * R[b][0] + R[a][1] * d[1] * R[b][1] + R[a][2] * d[2] * R[b][2];
  }
}

template <typename T>
struct ThetaSet {
  const T* p[6];
};
template <typename T>
struct ThetaOut {
  T* p[6];
};

// One stage: out = c0 Theta_n + c1 (Theta_in + dt RH(Theta_in)); LAST also writes tau_p from
// the new Theta. Theta_n and out may be the same arrays (each thread reads Theta_n at its own
// cell only; neighbours are read from Theta_in).
template <typename T, bool LAST, bool WENO>
__global__ void __launch_bounds__(kBlock)
    k_lcr_stage(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
                ThetaSet<T> thn, ThetaSet<T> thin, ThetaOut<T> thout, ThetaOut<T> tauout, int nx,
                int ny, int nz, T ihx, T ihy, T ihz, double dt, double inv_wi, double alpha,
                double c0, double c1, double tau_scale, Walls<T> wl) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  const int k = bz;
  const int id = (k * ny + j) * nx + i;
  const Coarse<T> U{u, nx, ny, nz}, V{v, nx, ny, nz}, Wf{w, nx, ny, nz};
  // eigenframe of Theta_in at this cell first (the neighbours are needed only for advection)
  double th6[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) th6[m] = (double)thin.p[m][id];
  double A[3][3], R[3][3];
  unpack6(th6, A);
  jacobi3(A, R);
  const double th[3] = {A[0][0], A[1][1], A[2][2]};
  // L[a][b] = du_b/dx_a, so K_ij = L[j][i]
  T L[3][3];
  velocity_gradient(U, V, Wf, k, j, i, nz, ihx, ihy, ihz, L, wl);
  double K[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) K[a][b] = (double)L[b][a];
  // M = R^T K R
  double KR[3][3], M[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) KR[a][b] = K[a][0] * R[0][b] + K[a][1] * R[1][b] + K[a][2] * R[2][b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[a][b] = R[0][a] * KR[0][b] + R[1][a] * KR[1][b] + R[2][a] * KR[2][b];
  // eigenframe source: commutator (off-diagonal) + 2 diag(m) - relaxation / Wi (diagonal)
  double S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double rel = -expm1(-th[a]) * (1.0 + alpha * expm1(th[a]));
    S[a][a] = 2.0 * M[a][a] - inv_wi * rel;
  }
  S[0][1] = S[1][0] = commutator_entry(th[1] - th[0], M[0][1], M[1][0]);
  S[0][2] = S[2][0] = commutator_entry(th[2] - th[0], M[0][2], M[2][0]);
  S[1][2] = S[2][1] = commutator_entry(th[2] - th[1], M[1][2], M[2][1]);
  // back to the physical frame: R S R^T
  double RS[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) RS[a][b] = R[a][0] * S[0][b] + R[a][1] * S[1][b] + R[a][2] * S[2][b];
  const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
  // advection: -div(u Theta) in flux form, face-mean values, zero wall flux
  const T h = (T)0.5;
  const T uxp = U.at(k, j, i), uxm = U.at(k, j, i - 1);
  const T vyp = V.at(k, j, i), vym = V.at(k, j - 1, i);
  const T wzp = k < nz - 1 ? Wf.at(k, j, i) : (T)0, wzm = k > 0 ? Wf.at(k - 1, j, i) : (T)0;
  double out[6];
  const WenoOffsets<T> wo(k, j, WENO ? i : 0, nx, ny, nz);
  const NbrOffsets<T> no(k, j, i, nx, ny, nz);
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const T t0 = (T)th6[m];
    double adv;
    if (WENO) {
      // WENO-Z face values, three cells either way, mirrored beyond the walls
      adv = (double)wo.advection(thin.p[m], uxm, uxp, vym, vyp, wzm, wzp, ihx, ihy, ihz);
    } else {
      const T* q = thin.p[m];
      const T fxp = uxp * h * (t0 + ld_at(q, no.xp));
      const T fxm = uxm * h * (ld_at(q, no.xm) + t0);
      const T fyp = vyp * h * (t0 + ld_at(q, no.yp));
      const T fym = vym * h * (ld_at(q, no.ym) + t0);
      const T fzp = k < nz - 1 ? wzp * h * (t0 + ld_at(q, no.zp)) : (T)0;
      const T fzm = k > 0 ? wzm * h * (ld_at(q, no.zm) + t0) : (T)0;
      adv = -(double)((fxp - fxm) * ihx + (fyp - fym) * ihy + (fzp - fzm) * ihz);
    }
    const int a = pa[m], b = pb[m];
    const double src = RS[a][0] * R[b][0] + RS[a][1] * R[b][1] + RS[a][2] * R[b][2];
    out[m] = c0 * (double)thn.p[m][id] + c1 * (th6[m] + dt * (adv + src));
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) thout.p[m][id] = (T)out[m];
  if (LAST) {
    // tau_p = (1 - beta)/Wi (c - I), c - I = V diag(expm1(theta)) V^T for the eigenpairs of the
    // stored Theta^{n+1}. It differs from Theta_in by O(dt), so its Jacobi starts in the
    // eigenframe R of Theta_in: B = R^T Theta^{n+1} R is nearly diagonal, V = R Q.
    double o6[6], Tn[3][3], TR[3][3], B[3][3], Q[3][3], Vq[3][3];
#pragma unroll
    for (int m = 0; m < 6; ++m) o6[m] = (double)(T)out[m];
    unpack6(o6, Tn);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) TR[a][b] = Tn[a][0] * R[0][b] + Tn[a][1] * R[1][b] + Tn[a][2] * R[2][b];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) B[a][b] = B[b][a] = R[0][a] * TR[0][b] + R[1][a] * TR[1][b] + R[2][a] * TR[2][b];
    jacobi3(B, Q);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) Vq[a][b] = R[a][0] * Q[0][b] + R[a][1] * Q[1][b] + R[a][2] * Q[2][b];
    const double e[3] = {expm1(B[0][0]), expm1(B[1][1]), expm1(B[2][2])};
    double cm[6];
    rdr6(Vq, e, cm);
#pragma unroll
    for (int m = 0; m < 6; ++m) tauout.p[m][id] = (T)(tau_scale * cm[m]);
  }
}

}  // namespace

template <typename T>
hipError_t launch_lcr_stage(const Dims& c, const StepConsts& k, const T* u, const T* v, const T* w,
                            const T* const theta_n[6], const T* const theta_in[6], T* const theta_out[6],
                            T* const tau_out[6], double c0, double c1, hipStream_t st) {
  ThetaSet<T> tn, ti;
  ThetaOut<T> to, ta;
  for (int m = 0; m < 6; ++m) {
    tn.p[m] = theta_n[m];
    ti.p[m] = theta_in[m];
    to.p[m] = theta_out[m];
    ta.p[m] = tau_out ? tau_out[m] : nullptr;
  }
  const Launch3 L = launch3(c.nx, c.ny, c.nz);
  const double tau_scale = (1.0 - k.beta) / k.wi;
  const Walls<T> wl = walls_of<T>(k);
#define DRPF_LCR(LAST, WENO)                                                                      \
  hipLaunchKernelGGL((k_lcr_stage<T, LAST, WENO>), L.grid, L.block, 0, st, u, v, w, tn, ti, to, ta, c.nx, \
                     c.ny, c.nz, (T)c.ihx, (T)c.ihy, (T)c.ihz, k.dt, k.inv_wi, k.giesekus, c0, c1,      \
                     tau_scale, wl)
  if (k.advection == 1) {
    if (tau_out) DRPF_LCR(true, true); else DRPF_LCR(false, true);
  } else {
    if (tau_out) DRPF_LCR(true, false); else DRPF_LCR(false, false);
  }
#undef DRPF_LCR
  return hipGetLastError();
}

#define INST(T)                                                                                          \
  template hipError_t launch_lcr_stage<T>(const Dims&, const StepConsts&, const T*, const T*, const T*, \
                                          const T* const[6], const T* const[6], T* const[6], T* const[6], \
                                          double, double, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
