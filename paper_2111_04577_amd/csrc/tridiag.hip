// Wall-normal pass of the constant-coefficient solver: after the x and y transforms every
// Fourier mode (kx, ky) leaves a tridiagonal system across the walls,
//   (a x_{k-1} + (lam_xy - 2a) x_k + a x_{k+1}) * coeff - shift x_k = d_k,
// whose end rows carry the wall rule (Neumann ghost = adjacent, no-slip ghost = -adjacent,
// or the z-face form with zero wall values). One thread owns one mode and runs the Thomas
// elimination down the z column; consecutive threads own consecutive kx, so each z step of
// a wavefront is one contiguous load. Elimination factors go to a per-mode scratch column.
//
// Passes:
//   zpass_ch  -- the two Helmholtz operators of the Dong splitting (eqs. NS26-NS27),
//                (L - c_psi) then (L + alpha), applied back to back per mode.
//   zpass_ns  -- the three velocity Helmholtz solves of eq. NS36, the divergence of the
//                predicted velocity, the pressure-increment Poisson solve of eq. NS37 in
//                FP64 with the (0,0) mode pinned and its mean removed, and the correction
//                of eqs. NS38 (all per mode, in spectral x/y space).
//   zpass_helmholtz -- one generic solve (the drpf_helmholtz_solve entry point).
#include "kernels.hpp"

namespace drpf {

namespace {

constexpr int kZBlock = 128;

// Thomas elimination in place on a strided complex column. Arithmetic in A (double for the
// FP64 islands), storage in T. Rows: b0 (first), bi (interior), bn (last), off-diagonal a.
// Pivot factors c'_k go to piv[k * pstride]. `scale` multiplies the right-hand side.
template <typename T, typename A>
__device__ __forceinline__ void thomas(cx<T>* x, size_t stride, int n, A a, A b0, A bi, A bn,
                                       A* piv, size_t pstride, A scale) {
  A cp = 0;
  cx<A> dp = mk<A>(0, 0);
  for (int k = 0; k < n; ++k) {
    const A b = k == 0 ? b0 : (k == n - 1 ? bn : bi);
    const A inv = (A)1 / (b - a * cp);
    cx<A> d = widen<A>(x[k * stride]);
    d = mk<A>(scale * d.re - a * dp.re, scale * d.im - a * dp.im);
    dp = inv * d;
    cp = a * inv;
    piv[k * pstride] = cp;
    x[k * stride] = mk<T>((T)dp.re, (T)dp.im);
  }
  cx<A> xn = dp;
  for (int k = n - 2; k >= 0; --k) {
    const cx<A> dk = widen<A>(x[k * stride]);
    const A c = piv[k * pstride];
    xn = mk<A>(dk.re - c * xn.re, dk.im - c * xn.im);
    x[k * stride] = mk<T>((T)xn.re, (T)xn.im);
  }
}

// Same elimination on a column kept in double precision registers via a double scratch
// column `col` (used by the FP64 Poisson island so that FP32 storage never rounds the
// intermediate elimination values).
__device__ __forceinline__ void thomas_d(double* colre, double* colim, size_t cstride, int n,
                                         double a, double b0, double bi, double bn, double* piv,
                                         size_t pstride) {
  double cp = 0, dre = 0, dim = 0;
  for (int k = 0; k < n; ++k) {
    const double b = k == 0 ? b0 : (k == n - 1 ? bn : bi);
    const double inv = 1.0 / (b - a * cp);
    dre = (colre[k * cstride] - a * dre) * inv;
    dim = (colim[k * cstride] - a * dim) * inv;
    cp = a * inv;
    piv[k * pstride] = cp;
    colre[k * cstride] = dre;
    colim[k * cstride] = dim;
  }
  for (int k = n - 2; k >= 0; --k) {
    const double c = piv[k * pstride];
    dre = colre[k * cstride] - c * dre;
    dim = colim[k * cstride] - c * dim;
    colre[k * cstride] = dre;
    colim[k * cstride] = dim;
  }
}

template <typename T>
__global__ void __launch_bounds__(kZBlock)
    k_zpass_helmholtz(cx<T>* __restrict__ S, double* __restrict__ piv, int P, int Ny, int Nz,
                      const double* __restrict__ lamx, const double* __restrict__ lamy, double hz,
                      int bc, double coeff, double shift, double scale) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int lines = P * Ny;
  if (l >= lines) return;
  const int ky = l / P;
  const int kx = l - ky * P;
  const size_t stride = (size_t)lines;
  const double a = coeff / (hz * hz);
  const double dxy = coeff * (lamx[kx] + lamy[ky]) - shift;
  cx<T>* col = S + l;
  double* pv = piv + l;
  if (bc == 0) {
    if (shift == 0.0 && kx == 0 && ky == 0) {
      // singular Neumann Poisson mode: pin x_0 = 0, solve rows 1..Nz-1, remove the mean
      col[0] = mk<T>(0, 0);
      thomas<T, double>(col + stride, stride, Nz - 1, a, dxy - 2 * a, dxy - 2 * a, dxy - a,
                        pv + stride, stride, scale);
      double mre = 0, mim = 0;
      for (int k = 0; k < Nz; ++k) {
        mre += (double)col[k * stride].re;
        mim += (double)col[k * stride].im;
      }
      mre /= Nz;
      mim /= Nz;
      for (int k = 0; k < Nz; ++k) {
        const cx<T> v = col[k * stride];
        col[k * stride] = mk<T>((T)((double)v.re - mre), (T)((double)v.im - mim));
      }
    } else {
      thomas<T, double>(col, stride, Nz, a, dxy - a, dxy - 2 * a, dxy - a, pv, stride, scale);
    }
  } else if (bc == 1) {
    thomas<T, double>(col, stride, Nz, a, dxy - 3 * a, dxy - 2 * a, dxy - 3 * a, pv, stride, scale);
  } else {
    thomas<T, double>(col, stride, Nz - 1, a, dxy - 2 * a, dxy - 2 * a, dxy - 2 * a, pv, stride,
                      scale);
    col[(Nz - 1) * stride] = mk<T>(0, 0);
  }
}

template <typename T>
__global__ void __launch_bounds__(kZBlock)
    k_zpass_ch(cx<T>* __restrict__ S, T* __restrict__ piv, int P, int Ny, int Nz,
               const double* __restrict__ lamx, const double* __restrict__ lamy, double hz,
               double c_psi, double alpha, double scale) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int lines = P * Ny;
  if (l >= lines) return;
  const int ky = l / P;
  const int kx = l - ky * P;
  const size_t stride = (size_t)lines;
  const T a = (T)(1.0 / (hz * hz));
  const double lxy = lamx[kx] + lamy[ky];
  cx<T>* col = S + l;
  T* pv = piv + l;
  // (L_N - c_psi) Psi' = R
  {
    const T bi = (T)(lxy - 2.0 / (hz * hz) - c_psi);
    const T be = (T)(lxy - 1.0 / (hz * hz) - c_psi);
    thomas<T, T>(col, stride, Nz, a, be, bi, be, pv, stride, (T)scale);
  }
  // (L_N + alpha) phi = Psi'
  {
    const T bi = (T)(lxy - 2.0 / (hz * hz) + alpha);
    const T be = (T)(lxy - 1.0 / (hz * hz) + alpha);
    thomas<T, T>(col, stride, Nz, a, be, bi, be, pv, stride, (T)1);
  }
}

// NS spectral pass. spec holds four fields of Nz*Ny*P complex each: r_u, r_v, r_w on entry
// (fields 0-2); on exit u^{n+1}, v^{n+1}, w^{n+1} and the pressure increment p' (field 3).
// pivd: double scratch with room for 3 columns (pivots, p' real and imaginary parts) per mode.
template <typename T>
__global__ void __launch_bounds__(kZBlock)
    k_zpass_ns(cx<T>* __restrict__ spec, double* __restrict__ pivd, int P, int Ny, int Nz,
               const double* __restrict__ lamx, const double* __restrict__ lamy,
               const double* __restrict__ phx, const double* __restrict__ phy, double hx,
               double hy, double hz, double nu_m, double g_dt, double g_rho_dt, double scale) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int lines = P * Ny;
  if (l >= lines) return;
  const int ky = l / P;
  const int kx = l - ky * P;
  const size_t stride = (size_t)lines;
  const size_t fsz = (size_t)lines * Nz;
  cx<T>* U = spec + l;
  cx<T>* V = spec + fsz + l;
  cx<T>* W = spec + 2 * fsz + l;
  cx<T>* Pp = spec + 3 * fsz + l;
  double* piv = pivd + l;
  double* pre = pivd + fsz + l;
  double* pim = pivd + 2 * fsz + l;
  const double lxy = lamx[kx] + lamy[ky];
  // ---- velocity Helmholtz solves (nu_m L - gamma0/dt) u~ = r
  const double a = nu_m / (hz * hz);
  const double bi = nu_m * lxy - 2 * a - g_dt;
  const double be = nu_m * lxy - 3 * a - g_dt;
  thomas<T, double>(U, stride, Nz, a, be, bi, be, piv, stride, scale);
  if (Ny > 1) thomas<T, double>(V, stride, Nz, a, be, bi, be, piv, stride, scale);
  thomas<T, double>(W, stride, Nz - 1, a, bi, bi, bi, piv, stride, scale);
  W[(Nz - 1) * stride] = mk<T>(0, 0);
  // ---- divergence at centres, spectral in x/y: D_x = (1 - e^{-i th_x}) / hx
  const double cxr = phx[2 * kx], cxi = phx[2 * kx + 1];
  const double cyr = phy[2 * ky], cyi = phy[2 * ky + 1];
  // 1 - e^{-i th} = (1 - cos th) + i sin th
  const double dxr = (1.0 - cxr) / hx, dxi = cxi / hx;
  const double dyr = (1.0 - cyr) / hy, dyi = cyi / hy;
  double wre_prev = 0, wim_prev = 0;
  for (int k = 0; k < Nz; ++k) {
    const cx<double> u = widen<double>(U[k * stride]);
    const cx<double> v = Ny > 1 ? widen<double>(V[k * stride]) : mk<double>(0, 0);
    const cx<double> w = widen<double>(W[k * stride]);
    double re = dxr * u.re - dxi * u.im + dyr * v.re - dyi * v.im + (w.re - wre_prev) / hz;
    double im = dxr * u.im + dxi * u.re + dyr * v.im + dyi * v.re + (w.im - wim_prev) / hz;
    wre_prev = w.re;
    wim_prev = w.im;
    pre[k * stride] = g_rho_dt * re;
    pim[k * stride] = g_rho_dt * im;
  }
  // ---- FP64 Poisson (Neumann) for p'
  const double ap = 1.0 / (hz * hz);
  if (kx == 0 && ky == 0) {
    pre[0] = 0;
    pim[0] = 0;
    thomas_d(pre + stride, pim + stride, stride, Nz - 1, ap, lxy - 2 * ap, lxy - 2 * ap, lxy - ap,
             piv + stride, stride);
    double mre = 0, mim = 0;
    for (int k = 0; k < Nz; ++k) {
      mre += pre[k * stride];
      mim += pim[k * stride];
    }
    mre /= Nz;
    mim /= Nz;
    for (int k = 0; k < Nz; ++k) {
      pre[k * stride] -= mre;
      pim[k * stride] -= mim;
    }
  } else {
    thomas_d(pre, pim, stride, Nz, ap, lxy - ap, lxy - 2 * ap, lxy - ap, piv, stride);
  }
  // ---- correction u = u~ - c grad p', G_x = (e^{i th_x} - 1) / hx
  const double c = 1.0 / g_rho_dt;
  const double gxr = (cxr - 1.0) / hx, gxi = cxi / hx;
  const double gyr = (cyr - 1.0) / hy, gyi = cyi / hy;
  for (int k = 0; k < Nz; ++k) {
    const double pr = pre[k * stride], pi = pim[k * stride];
    const cx<double> u = widen<double>(U[k * stride]);
    U[k * stride] = mk<T>((T)(u.re - c * (gxr * pr - gxi * pi)), (T)(u.im - c * (gxr * pi + gxi * pr)));
    if (Ny > 1) {
      const cx<double> v = widen<double>(V[k * stride]);
      V[k * stride] = mk<T>((T)(v.re - c * (gyr * pr - gyi * pi)), (T)(v.im - c * (gyr * pi + gyi * pr)));
    }
    if (k < Nz - 1) {
      const double qr = pre[(k + 1) * stride], qi = pim[(k + 1) * stride];
      const cx<double> w = widen<double>(W[k * stride]);
      W[k * stride] = mk<T>((T)(w.re - c * (qr - pr) / hz), (T)(w.im - c * (qi - pi) / hz));
    }
    Pp[k * stride] = mk<T>((T)pr, (T)pi);
  }
}

}  // namespace

template <typename T>
hipError_t launch_zpass_helmholtz(const Dims& d, const Tables<T>& tb, cx<T>* spec, double* piv,
                                  int bc, double coeff, double shift, double scale, hipStream_t st) {
  const int lines = d.lines();
  hipLaunchKernelGGL(k_zpass_helmholtz<T>, dim3((lines + kZBlock - 1) / kZBlock), dim3(kZBlock), 0,
                     st, spec, piv, d.pitch, d.ny, d.nz, tb.lam_x, tb.lam_y, d.hz, bc, coeff, shift,
                     scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zpass_ch(const Dims& d, const Tables<T>& tb, cx<T>* spec, double* piv,
                           double c_psi, double alpha, double scale, hipStream_t st) {
  const int lines = d.lines();
  hipLaunchKernelGGL(k_zpass_ch<T>, dim3((lines + kZBlock - 1) / kZBlock), dim3(kZBlock), 0, st,
                     spec, reinterpret_cast<T*>(piv), d.pitch, d.ny, d.nz, tb.lam_x, tb.lam_y, d.hz,
                     c_psi, alpha, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zpass_ns(const Dims& d, const Tables<T>& tb, cx<T>* spec4, double* piv,
                           const StepConsts& c, double scale, hipStream_t st) {
  const int lines = d.lines();
  hipLaunchKernelGGL(k_zpass_ns<T>, dim3((lines + kZBlock - 1) / kZBlock), dim3(kZBlock), 0, st,
                     spec4, piv, d.pitch, d.ny, d.nz, tb.lam_x, tb.lam_y, tb.ph_x, tb.ph_y, d.hx, d.hy,
                     d.hz, c.nu_m, c.gamma0 / c.dt, c.gamma0 * c.rho0 / c.dt, scale);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_zpass_helmholtz<T>(const Dims&, const Tables<T>&, cx<T>*, double*,  \
                                                int, double, double, double, hipStream_t);       \
  template hipError_t launch_zpass_ch<T>(const Dims&, const Tables<T>&, cx<T>*, double*, double, \
                                         double, double, hipStream_t);                           \
  template hipError_t launch_zpass_ns<T>(const Dims&, const Tables<T>&, cx<T>*, double*,         \
                                         const StepConsts&, double, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
