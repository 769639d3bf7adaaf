// Coarse-grid (flow) stencils.
//
//   momentum_rhs   -- right-hand side r of the velocity Helmholtz equations of eq. NS36,
//                     (nu_m L - gamma0/dt) u~ = r, for the three components at their own
//                     faces. r collects -u_hat/dt (eq. NS35), the conservative central
//                     advection of u*, the diffusive-flux term J.grad(u*)/rho, the split
//                     pressure gradient (1/rho0) grad p^n + (1/rho - 1/rho0) grad p*, the
//                     explicit nu_m L u*, the polymer divergence of the second approach
//                     (eq. NS12, drop = polymer phase), the variable-viscosity stress
//                     divergence, the capillary force G grad(phi) and the body force.
//   polymer_stage  -- one stage of the second-order TVD Runge-Kutta update of the polymer
//                     stress (eqs. NS42, NS44) for the Oldroyd-B law in stress form.
//
// Staggering: u[k][j][i] at ((i+1) hx, (j+.5) hy, (k+.5) hz), v at (i+.5, j+1, k+.5),
// w at (i+.5, j+.5, k+1) with w[nz-1] the top wall; centres at (i+.5, j+.5, k+.5).
// Wall rules: no-slip ghost = -adjacent for u, v; w = 0 on the walls; Neumann ghost for
// centred scalars (G, tau).
#include "kernels.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;

template <typename T>
struct Field {
  const T* a;
  const T* b;   // level n-1 (extrapolation) or null
  int nx, ny, nz, first;
  // extrapolated value (u* = 2 u^n - u^{n-1}, or u^n on the first step), in-range k
  __device__ __forceinline__ double s(int k, int j, int i) const {
    const size_t id = ((size_t)k * ny + wrap(j, ny)) * nx + wrap(i, nx);
    return (first || b == nullptr) ? (double)a[id] : 2.0 * (double)a[id] - (double)b[id];
  }
  __device__ __forceinline__ double n(int k, int j, int i) const {
    return (double)a[((size_t)k * ny + wrap(j, ny)) * nx + wrap(i, nx)];
  }
  // cell-centred-in-z velocity with no-slip ghosts
  __device__ __forceinline__ double sd(int k, int j, int i) const {
    if (k < 0) return -s(0, j, i);
    if (k >= nz) return -s(nz - 1, j, i);
    return s(k, j, i);
  }
  // z-face velocity: index -1 is the bottom wall, nz-1 the top wall (stored 0), beyond 0
  __device__ __forceinline__ double sw(int k, int j, int i) const {
    if (k < 0 || k >= nz - 1) return 0.0;
    return s(k, j, i);
  }
  // centred scalar with Neumann ghosts
  __device__ __forceinline__ double sn(int k, int j, int i) const {
    return s(min(max(k, 0), nz - 1), j, i);
  }
  __device__ __forceinline__ double nn(int k, int j, int i) const {
    return n(min(max(k, 0), nz - 1), j, i);
  }
};

template <typename T>
struct Coarse {
  const T* a;
  int nx, ny, nz;
  __device__ __forceinline__ double at(int k, int j, int i) const {
    return (double)a[((size_t)k * ny + wrap(j, ny)) * nx + wrap(i, nx)];
  }
  __device__ __forceinline__ double atn(int k, int j, int i) const {
    return at(min(max(k, 0), nz - 1), j, i);
  }
};

// z-edge arrays (nz + 1 layers): layer m is the edge at z = m hz
template <typename T>
struct ZEdge {
  const T* a;
  int nx, ny;
  __device__ __forceinline__ double at(int m, int j, int i) const {
    return (double)a[((size_t)m * ny + wrap(j, ny)) * nx + wrap(i, nx)];
  }
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_momentum_rhs(NsIn<T> in, Restricted<T> R, T* __restrict__ ru, T* __restrict__ rv,
                   T* __restrict__ rw, int nx, int ny, int nz, double hx, double hy, double hz,
                   StepConsts c) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)nx * ny * nz;
  if (id >= n) return;
  const int i = (int)(id % nx);
  const int j = (int)((id / nx) % ny);
  const int k = (int)(id / ((size_t)nx * ny));
  const int f = c.first;
  const Field<T> U{in.un, in.unm1, nx, ny, nz, f}, V{in.vn, in.vnm1, nx, ny, nz, f},
      W{in.wn, in.wnm1, nx, ny, nz, f}, P{in.pn, in.pnm1, nx, ny, nz, f};
  const Field<T> Pn{in.pn, nullptr, nx, ny, nz, 1};
  const Coarse<T> Gc{R.G_c, nx, ny, nz}, phic{R.phi_c, nx, ny, nz}, muc{R.mu_c, nx, ny, nz},
      muxy{R.mu_xy, nx, ny, nz};
  const ZEdge<T> muxz{R.mu_xz, nx, ny}, muyz{R.mu_yz, nx, ny};
  const double ihx = 1.0 / hx, ihy = 1.0 / hy, ihz = 1.0 / hz;
  const double dt = c.dt;
  const double inv_re = 1.0 / c.re;
  const double ir0 = 1.0 / c.rho0;

  // hat (eq. NS31) of a field at an in-range index
  auto hat = [&](const T* a, const T* b, size_t idx) -> double {
    return f ? (double)a[idx] : 2.0 * (double)a[idx] - 0.5 * (double)b[idx];
  };
  // J = -c_j grad G at centre (k, j, i): 2h central differences, Neumann in z
  auto Jc = [&](int kk, int jj, int ii, double* J) {
    J[0] = -c.c_j * (Gc.at(kk, jj, ii + 1) - Gc.at(kk, jj, ii - 1)) * 0.5 * ihx;
    J[1] = -c.c_j * (Gc.at(kk, jj + 1, ii) - Gc.at(kk, jj - 1, ii)) * 0.5 * ihy;
    J[2] = -c.c_j * (Gc.atn(kk + 1, jj, ii) - Gc.atn(kk - 1, jj, ii)) * 0.5 * ihz;
  };
  // polymer weight T = (1 + phi_c)/2 * tau*, Neumann ghosts
  auto Tp = [&](int comp, int kk, int jj, int ii) -> double {
    const Field<T> t{in.taun[comp], in.taunm1[comp], nx, ny, nz, f};
    return 0.5 * (1.0 + phic.atn(kk, jj, ii)) * t.sn(kk, jj, ii);
  };
  const bool ve = in.viscoelastic != 0;
  const double ax[3] = {c.ax, c.ay, c.az};

  // ------------------------------------------------------------------ u at x face (i,j,k)
  {
    const double u0 = U.s(k, j, i);
    // advection
    const double ucr = 0.5 * (u0 + U.s(k, j, i + 1)), ucl = 0.5 * (U.s(k, j, i - 1) + u0);
    double adv = (ucr * ucr - ucl * ucl) * ihx;
    const double fyp = 0.5 * (V.s(k, j, i) + V.s(k, j, i + 1)) * 0.5 * (u0 + U.s(k, j + 1, i));
    const double fym = 0.5 * (V.s(k, j - 1, i) + V.s(k, j - 1, i + 1)) * 0.5 * (U.s(k, j - 1, i) + u0);
    adv += (fyp - fym) * ihy;
    const double fzp = 0.5 * (W.sw(k, j, i) + W.sw(k, j, i + 1)) * 0.5 * (u0 + U.sd(k + 1, j, i));
    const double fzm = 0.5 * (W.sw(k - 1, j, i) + W.sw(k - 1, j, i + 1)) * 0.5 * (U.sd(k - 1, j, i) + u0);
    adv += (fzp - fzm) * ihz;
    // J . grad u*
    double Ja[3], Jb[3];
    Jc(k, j, i, Ja);
    Jc(k, j, i + 1, Jb);
    const double jgu = 0.5 * (Ja[0] + Jb[0]) * (U.s(k, j, i + 1) - U.s(k, j, i - 1)) * 0.5 * ihx +
                       0.5 * (Ja[1] + Jb[1]) * (U.s(k, j + 1, i) - U.s(k, j - 1, i)) * 0.5 * ihy +
                       0.5 * (Ja[2] + Jb[2]) * (U.sd(k + 1, j, i) - U.sd(k - 1, j, i)) * 0.5 * ihz;
    // viscous stress divergence
    double vis = (2 * muc.at(k, j, i + 1) * (U.s(k, j, i + 1) - u0) * ihx -
                  2 * muc.at(k, j, i) * (u0 - U.s(k, j, i - 1)) * ihx) * ihx;
    const double sxyp = muxy.at(k, j, i) * ((U.s(k, j + 1, i) - u0) * ihy + (V.s(k, j, i + 1) - V.s(k, j, i)) * ihx);
    const double sxym = muxy.at(k, j - 1, i) * ((u0 - U.s(k, j - 1, i)) * ihy + (V.s(k, j - 1, i + 1) - V.s(k, j - 1, i)) * ihx);
    vis += (sxyp - sxym) * ihy;
    const double sxzp = muxz.at(k + 1, j, i) * ((U.sd(k + 1, j, i) - u0) * ihz + (W.sw(k, j, i + 1) - W.sw(k, j, i)) * ihx);
    const double sxzm = muxz.at(k, j, i) * ((u0 - U.sd(k - 1, j, i)) * ihz + (W.sw(k - 1, j, i + 1) - W.sw(k - 1, j, i)) * ihx);
    vis += (sxzp - sxzm) * ihz;
    // polymer divergence
    double pol = 0;
    if (ve) {
      pol = (Tp(0, k, j, i + 1) - Tp(0, k, j, i)) * ihx;
      auto txy = [&](int jj) {
        return 0.25 * (Tp(3, k, jj, i) + Tp(3, k, jj, i + 1) + Tp(3, k, jj + 1, i) + Tp(3, k, jj + 1, i + 1));
      };
      pol += (txy(j) - txy(j - 1)) * ihy;
      auto txz = [&](int kk) {  // edge between centres kk and kk+1
        return 0.25 * (Tp(4, kk, j, i) + Tp(4, kk, j, i + 1) + Tp(4, kk + 1, j, i) + Tp(4, kk + 1, j, i + 1));
      };
      pol += (txz(k) - txz(k - 1)) * ihz;
    }
    const double ri = (double)R.ri_x[id];
    const double gpn = (Pn.n(k, j, i + 1) - Pn.n(k, j, i)) * ihx;
    const double gps = (P.s(k, j, i + 1) - P.s(k, j, i)) * ihx;
    const double cap = (double)R.G_x[id] * (phic.at(k, j, i + 1) - phic.at(k, j, i)) * ihx;
    const double lap = (U.s(k, j, i + 1) - 2 * u0 + U.s(k, j, i - 1)) * ihx * ihx +
                       (U.s(k, j + 1, i) - 2 * u0 + U.s(k, j - 1, i)) * ihy * ihy +
                       (U.sd(k + 1, j, i) - 2 * u0 + U.sd(k - 1, j, i)) * ihz * ihz;
    const double r = -hat(in.un, in.unm1, id) / dt + adv + ri * jgu + gpn * ir0 + (ri - ir0) * gps +
                     c.nu_m * lap - inv_re * ri * pol - inv_re * ri * vis - c.k_sigma * ri * cap - ax[0];
    ru[id] = (T)r;
  }
  // ------------------------------------------------------------------ v at y face (i,j,k)
  {
    const double v0 = V.s(k, j, i);
    const double vcu = 0.5 * (v0 + V.s(k, j + 1, i)), vcl = 0.5 * (V.s(k, j - 1, i) + v0);
    double adv = (vcu * vcu - vcl * vcl) * ihy;
    const double fxp = 0.5 * (U.s(k, j, i) + U.s(k, j + 1, i)) * 0.5 * (v0 + V.s(k, j, i + 1));
    const double fxm = 0.5 * (U.s(k, j, i - 1) + U.s(k, j + 1, i - 1)) * 0.5 * (V.s(k, j, i - 1) + v0);
    adv += (fxp - fxm) * ihx;
    const double fzp = 0.5 * (W.sw(k, j, i) + W.sw(k, j + 1, i)) * 0.5 * (v0 + V.sd(k + 1, j, i));
    const double fzm = 0.5 * (W.sw(k - 1, j, i) + W.sw(k - 1, j + 1, i)) * 0.5 * (V.sd(k - 1, j, i) + v0);
    adv += (fzp - fzm) * ihz;
    double Ja[3], Jb[3];
    Jc(k, j, i, Ja);
    Jc(k, j + 1, i, Jb);
    const double jgv = 0.5 * (Ja[0] + Jb[0]) * (V.s(k, j, i + 1) - V.s(k, j, i - 1)) * 0.5 * ihx +
                       0.5 * (Ja[1] + Jb[1]) * (V.s(k, j + 1, i) - V.s(k, j - 1, i)) * 0.5 * ihy +
                       0.5 * (Ja[2] + Jb[2]) * (V.sd(k + 1, j, i) - V.sd(k - 1, j, i)) * 0.5 * ihz;
    double vis = (2 * muc.at(k, j + 1, i) * (V.s(k, j + 1, i) - v0) * ihy -
                  2 * muc.at(k, j, i) * (v0 - V.s(k, j - 1, i)) * ihy) * ihy;
    const double sxyp = muxy.at(k, j, i) * ((U.s(k, j + 1, i) - U.s(k, j, i)) * ihy + (V.s(k, j, i + 1) - v0) * ihx);
    const double sxym = muxy.at(k, j, i - 1) * ((U.s(k, j + 1, i - 1) - U.s(k, j, i - 1)) * ihy + (v0 - V.s(k, j, i - 1)) * ihx);
    vis += (sxyp - sxym) * ihx;
    const double syzp = muyz.at(k + 1, j, i) * ((V.sd(k + 1, j, i) - v0) * ihz + (W.sw(k, j + 1, i) - W.sw(k, j, i)) * ihy);
    const double syzm = muyz.at(k, j, i) * ((v0 - V.sd(k - 1, j, i)) * ihz + (W.sw(k - 1, j + 1, i) - W.sw(k - 1, j, i)) * ihy);
    vis += (syzp - syzm) * ihz;
    double pol = 0;
    if (ve) {
      auto txy = [&](int ii) {
        return 0.25 * (Tp(3, k, j, ii) + Tp(3, k, j, ii + 1) + Tp(3, k, j + 1, ii) + Tp(3, k, j + 1, ii + 1));
      };
      pol = (txy(i) - txy(i - 1)) * ihx;
      pol += (Tp(1, k, j + 1, i) - Tp(1, k, j, i)) * ihy;
      auto tyz = [&](int kk) {
        return 0.25 * (Tp(5, kk, j, i) + Tp(5, kk, j + 1, i) + Tp(5, kk + 1, j, i) + Tp(5, kk + 1, j + 1, i));
      };
      pol += (tyz(k) - tyz(k - 1)) * ihz;
    }
    const double ri = (double)R.ri_y[id];
    const double gpn = (Pn.n(k, j + 1, i) - Pn.n(k, j, i)) * ihy;
    const double gps = (P.s(k, j + 1, i) - P.s(k, j, i)) * ihy;
    const double cap = (double)R.G_y[id] * (phic.at(k, j + 1, i) - phic.at(k, j, i)) * ihy;
    const double lap = (V.s(k, j, i + 1) - 2 * v0 + V.s(k, j, i - 1)) * ihx * ihx +
                       (V.s(k, j + 1, i) - 2 * v0 + V.s(k, j - 1, i)) * ihy * ihy +
                       (V.sd(k + 1, j, i) - 2 * v0 + V.sd(k - 1, j, i)) * ihz * ihz;
    const double r = -hat(in.vn, in.vnm1, id) / dt + adv + ri * jgv + gpn * ir0 + (ri - ir0) * gps +
                     c.nu_m * lap - inv_re * ri * pol - inv_re * ri * vis - c.k_sigma * ri * cap - ax[1];
    rv[id] = (T)r;
  }
  // ------------------------------------------------------------------ w at z face (i,j,k)
  if (k == nz - 1) {
    rw[id] = (T)0;
  } else {
    const double w0 = W.sw(k, j, i);
    const double wcu = 0.5 * (w0 + W.sw(k + 1, j, i)), wcl = 0.5 * (W.sw(k - 1, j, i) + w0);
    double adv = (wcu * wcu - wcl * wcl) * ihz;
    const double fxp = 0.5 * (U.s(k, j, i) + U.s(k + 1, j, i)) * 0.5 * (w0 + W.sw(k, j, i + 1));
    const double fxm = 0.5 * (U.s(k, j, i - 1) + U.s(k + 1, j, i - 1)) * 0.5 * (W.sw(k, j, i - 1) + w0);
    adv += (fxp - fxm) * ihx;
    const double fyp = 0.5 * (V.s(k, j, i) + V.s(k + 1, j, i)) * 0.5 * (w0 + W.sw(k, j + 1, i));
    const double fym = 0.5 * (V.s(k, j - 1, i) + V.s(k + 1, j - 1, i)) * 0.5 * (W.sw(k, j - 1, i) + w0);
    adv += (fyp - fym) * ihy;
    double Ja[3], Jb[3];
    Jc(k, j, i, Ja);
    Jc(k + 1, j, i, Jb);
    const double jgw = 0.5 * (Ja[0] + Jb[0]) * (W.sw(k, j, i + 1) - W.sw(k, j, i - 1)) * 0.5 * ihx +
                       0.5 * (Ja[1] + Jb[1]) * (W.sw(k, j + 1, i) - W.sw(k, j - 1, i)) * 0.5 * ihy +
                       0.5 * (Ja[2] + Jb[2]) * (W.sw(k + 1, j, i) - W.sw(k - 1, j, i)) * 0.5 * ihz;
    double vis = (2 * muc.at(k + 1, j, i) * (W.sw(k + 1, j, i) - w0) * ihz -
                  2 * muc.at(k, j, i) * (w0 - W.sw(k - 1, j, i)) * ihz) * ihz;
    const double sxzp = muxz.at(k + 1, j, i) * ((W.sw(k, j, i + 1) - w0) * ihx + (U.s(k + 1, j, i) - U.s(k, j, i)) * ihz);
    const double sxzm = muxz.at(k + 1, j, i - 1) * ((w0 - W.sw(k, j, i - 1)) * ihx + (U.s(k + 1, j, i - 1) - U.s(k, j, i - 1)) * ihz);
    vis += (sxzp - sxzm) * ihx;
    const double syzp = muyz.at(k + 1, j, i) * ((W.sw(k, j + 1, i) - w0) * ihy + (V.s(k + 1, j, i) - V.s(k, j, i)) * ihz);
    const double syzm = muyz.at(k + 1, j - 1, i) * ((w0 - W.sw(k, j - 1, i)) * ihy + (V.s(k + 1, j - 1, i) - V.s(k, j - 1, i)) * ihz);
    vis += (syzp - syzm) * ihy;
    double pol = 0;
    if (ve) {
      auto txz = [&](int ii) {  // xz edge at z face k between x centres ii and ii+1
        return 0.25 * (Tp(4, k, j, ii) + Tp(4, k, j, ii + 1) + Tp(4, k + 1, j, ii) + Tp(4, k + 1, j, ii + 1));
      };
      auto tyz = [&](int jj) {
        return 0.25 * (Tp(5, k, jj, i) + Tp(5, k, jj + 1, i) + Tp(5, k + 1, jj, i) + Tp(5, k + 1, jj + 1, i));
      };
      pol = (txz(i) - txz(i - 1)) * ihx + (tyz(j) - tyz(j - 1)) * ihy +
            (Tp(2, k + 1, j, i) - Tp(2, k, j, i)) * ihz;
    }
    const double ri = (double)R.ri_z[id];
    const double gpn = (Pn.n(k + 1, j, i) - Pn.n(k, j, i)) * ihz;
    const double gps = (P.s(k + 1, j, i) - P.s(k, j, i)) * ihz;
    const double cap = (double)R.G_z[id] * (phic.at(k + 1, j, i) - phic.at(k, j, i)) * ihz;
    const double lap = (W.sw(k, j, i + 1) - 2 * w0 + W.sw(k, j, i - 1)) * ihx * ihx +
                       (W.sw(k, j + 1, i) - 2 * w0 + W.sw(k, j - 1, i)) * ihy * ihy +
                       (W.sw(k + 1, j, i) - 2 * w0 + W.sw(k - 1, j, i)) * ihz * ihz;
    const double r = -hat(in.wn, in.wnm1, id) / dt + adv + ri * jgw + gpn * ir0 + (ri - ir0) * gps +
                     c.nu_m * lap - inv_re * ri * pol - inv_re * ri * vis - c.k_sigma * ri * cap - ax[2];
    rw[id] = (T)r;
  }
}

// tau component index of the pair (a, b): xx, yy, zz, xy, xz, yz
__device__ __forceinline__ int tidx(int a, int b) {
  if (a == b) return a;
  const int s = a + b;  // 1: xy, 2: xz, 3: yz
  return 2 + s;
}

template <typename T>
struct TauSet {
  const T* p[6];
};
template <typename T>
struct TauOut {
  T* p[6];
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_polymer_stage(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
                    TauSet<T> tn, TauSet<T> tin, TauOut<T> tout, int nx, int ny, int nz, double hx,
                    double hy, double hz, double dt, double wi, double beta, double c0, double c1) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)nx * ny * nz;
  if (id >= n) return;
  const int i = (int)(id % nx);
  const int j = (int)((id / nx) % ny);
  const int k = (int)(id / ((size_t)nx * ny));
  const Coarse<T> U{u, nx, ny, nz}, V{v, nx, ny, nz}, Wf{w, nx, ny, nz};
  const double ihx = 1.0 / hx, ihy = 1.0 / hy, ihz = 1.0 / hz;
  auto wv = [&](int kk, int jj, int ii) -> double {
    return (kk < 0 || kk >= nz - 1) ? 0.0 : Wf.at(kk, jj, ii);
  };
  // cell-centred velocities
  auto uc = [&](int kk, int jj, int ii) -> double {
    if (kk < 0) return -0.5 * (U.at(0, jj, ii) + U.at(0, jj, ii - 1));
    if (kk >= nz) return -0.5 * (U.at(nz - 1, jj, ii) + U.at(nz - 1, jj, ii - 1));
    return 0.5 * (U.at(kk, jj, ii) + U.at(kk, jj, ii - 1));
  };
  auto vc = [&](int kk, int jj, int ii) -> double {
    if (kk < 0) return -0.5 * (V.at(0, jj, ii) + V.at(0, jj - 1, ii));
    if (kk >= nz) return -0.5 * (V.at(nz - 1, jj, ii) + V.at(nz - 1, jj - 1, ii));
    return 0.5 * (V.at(kk, jj, ii) + V.at(kk, jj - 1, ii));
  };
  auto wc = [&](int kk, int jj, int ii) -> double { return 0.5 * (wv(kk, jj, ii) + wv(kk - 1, jj, ii)); };
  // L[a][b] = d u_b / d x_a
  double L[3][3];
  L[0][0] = (U.at(k, j, i) - U.at(k, j, i - 1)) * ihx;
  L[1][1] = (V.at(k, j, i) - V.at(k, j - 1, i)) * ihy;
  L[2][2] = (wv(k, j, i) - wv(k - 1, j, i)) * ihz;
  L[0][1] = (vc(k, j, i + 1) - vc(k, j, i - 1)) * 0.5 * ihx;
  L[0][2] = (wc(k, j, i + 1) - wc(k, j, i - 1)) * 0.5 * ihx;
  L[1][0] = (uc(k, j + 1, i) - uc(k, j - 1, i)) * 0.5 * ihy;
  L[1][2] = (wc(k, j + 1, i) - wc(k, j - 1, i)) * 0.5 * ihy;
  L[2][0] = (uc(k + 1, j, i) - uc(k - 1, j, i)) * 0.5 * ihz;
  L[2][1] = (vc(k + 1, j, i) - vc(k - 1, j, i)) * 0.5 * ihz;
  double tau[6];
  for (int m = 0; m < 6; ++m) tau[m] = (double)tin.p[m][id];
  const double uxp = U.at(k, j, i), uxm = U.at(k, j, i - 1);
  const double vyp = V.at(k, j, i), vym = V.at(k, j - 1, i);
  const double wzp = wv(k, j, i), wzm = wv(k - 1, j, i);
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int m = 0; m < 6; ++m) {
    const int a = pairs[m][0], b = pairs[m][1];
    const Coarse<T> t{tin.p[m], nx, ny, nz};
    const double t0 = tau[m];
    const double fxp = uxp * 0.5 * (t0 + t.at(k, j, i + 1));
    const double fxm = uxm * 0.5 * (t.at(k, j, i - 1) + t0);
    const double fyp = vyp * 0.5 * (t0 + t.at(k, j + 1, i));
    const double fym = vym * 0.5 * (t.at(k, j - 1, i) + t0);
    const double fzp = k < nz - 1 ? wzp * 0.5 * (t0 + t.at(k + 1, j, i)) : 0.0;
    const double fzm = k > 0 ? wzm * 0.5 * (t.at(k - 1, j, i) + t0) : 0.0;
    double rh = -((fxp - fxm) * ihx + (fyp - fym) * ihy + (fzp - fzm) * ihz);
    for (int cc = 0; cc < 3; ++cc) rh += L[cc][a] * tau[tidx(cc, b)] + tau[tidx(a, cc)] * L[cc][b];
    rh += ((1.0 - beta) * (L[a][b] + L[b][a]) - t0) / wi;
    const double val = c0 * (double)tn.p[m][id] + c1 * (t0 + dt * rh);
    tout.p[m][id] = (T)val;
  }
}

}  // namespace

template <typename T>
hipError_t launch_momentum_rhs(const Dims& c, const StepConsts& k, NsIn<T> in, Restricted<T> r,
                               T* ru, T* rv, T* rw, hipStream_t st) {
  const size_t n = c.cells();
  hipLaunchKernelGGL(k_momentum_rhs<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     st, in, r, ru, rv, rw, c.nx, c.ny, c.nz, c.hx, c.hy, c.hz, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_polymer_stage(const Dims& c, const StepConsts& k, const T* u, const T* v,
                                const T* w, const T* const tau_n[6], const T* const tau_in[6],
                                T* const tau_out[6], double c0, double c1, hipStream_t st) {
  TauSet<T> tn, ti;
  TauOut<T> to;
  for (int m = 0; m < 6; ++m) {
    tn.p[m] = tau_n[m];
    ti.p[m] = tau_in[m];
    to.p[m] = tau_out[m];
  }
  const size_t n = c.cells();
  hipLaunchKernelGGL(k_polymer_stage<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     st, u, v, w, tn, ti, to, c.nx, c.ny, c.nz, c.hx, c.hy, c.hz, k.dt, k.wi, k.beta,
                     c0, c1);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_momentum_rhs<T>(const Dims&, const StepConsts&, NsIn<T>,             \
                                             Restricted<T>, T*, T*, T*, hipStream_t);             \
  template hipError_t launch_polymer_stage<T>(const Dims&, const StepConsts&, const T*, const T*, \
                                              const T*, const T* const[6], const T* const[6],     \
                                              T* const[6], double, double, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
