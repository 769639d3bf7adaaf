// Coarse-grid (flow) stencils.
//
//   momentum_rhs   -- right-hand side r of the velocity Helmholtz equations of eq. NS36,
//                     (nu_m L - gamma0/dt) u~ = r, for each component at its own faces.
//                     r collects -u_hat/dt (eq. NS35), the conservative central advection of
//                     u*, the diffusive-flux term J.grad(u*)/rho, the split pressure gradient
//                     (1/rho0) grad p^n + (1/rho - 1/rho0) grad p*, the explicit nu_m L u*,
//                     the polymer divergence of the second approach (eq. NS12, drop = polymer
//                     phase), the variable-viscosity stress divergence, the capillary force
//                     G grad(phi) and the body force. One launch covers the three components
//                     (uniform per block), interleaved layer by layer.
//   polymer_stage  -- one stage of the second-order TVD Runge-Kutta update of the polymer
//                     stress (eqs. NS42, NS44) for the Oldroyd-B law in stress form.
//
// Staggering: u[k][j][i] at ((i+1) hx, (j+.5) hy, (k+.5) hz), v at (i+.5, j+1, k+.5),
// w at (i+.5, j+.5, k+1) with w[nz-1] the top wall; centres at (i+.5, j+.5, k+.5).
// Wall rules: no-slip ghost = -adjacent for u, v; w = 0 on the walls; Neumann ghost for
// centred scalars (G, tau). Arithmetic in the storage type T.
#include "coarse.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_momentum_rhs(NsIn<T> in, Restricted<T> R, T* __restrict__ ru, T* __restrict__ rv,
                   T* __restrict__ rw, int nx, int ny, int nz, T ihx, T ihy, T ihz, StepConsts c) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  // blockIdx.z = 3 k + component: the three components of one layer are neighbouring tiles,
  // so each XCD's slab covers all of them and the shared inputs stay in its L2
  const int k = bz / 3;
  const int comp = bz - 3 * k;
  const int f = c.first;
  MomCtx<T> m{{in.un, in.unm1, nx, ny, nz, f},
              {in.vn, in.vnm1, nx, ny, nz, f},
              {in.wn, in.wnm1, nx, ny, nz, f},
              {in.pn, in.pnm1, nx, ny, nz, f},
              {in.pn, nullptr, nx, ny, nz, 1},
              {R.G_c, nx, ny, nz},
              {R.phi_c, nx, ny, nz},
              {R.mu_c, nx, ny, nz},
              {R.mu_xy, nx, ny, nz},
              {R.mu_xz, nx, ny},
              {R.mu_yz, nx, ny},
              in.taun,
              in.taunm1,
              R,
              nx, ny, nz, f, in.viscoelastic,
              ihx, ihy, ihz,
              (T)c.inv_dt, (T)c.inv_re, (T)c.inv_rho0, (T)c.nu_m, (T)c.k_sigma, (T)c.c_j};
  const int id = (k * ny + j) * nx + i;
  auto rhs = [&](const MomTerms<T>& t, T a) -> T {
    return -t.hat * m.inv_dt + t.adv + t.ri * t.jg + t.gpn * m.ir0 + (t.ri - m.ir0) * t.gps + m.nu_m * t.lap -
           m.inv_re * t.ri * t.pol - m.inv_re * t.ri * t.vis - m.k_sigma * t.ri * t.cap - a;
  };
  if (comp == 0) {
    ru[id] = rhs(mom_u(m, k, j, i, id), (T)c.ax);
  } else if (comp == 1) {
    rv[id] = rhs(mom_v(m, k, j, i, id), (T)c.ay);
  } else {
    rw[id] = k == nz - 1 ? (T)0 : rhs(mom_w(m, k, j, i, id), (T)c.az);
  }
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
                    TauSet<T> tn, TauSet<T> tin, TauOut<T> tout, int nx, int ny, int nz, T ihx,
                    T ihy, T ihz, T dt, T inv_wi, T one_m_beta, T c0, T c1) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  const int k = bz;
  const int id = (k * ny + j) * nx + i;
  const Coarse<T> U{u, nx, ny, nz}, V{v, nx, ny, nz}, Wf{w, nx, ny, nz};
  const T h = (T)0.5;
  // L[a][b] = d u_b / d x_a
  T L[3][3];
  velocity_gradient(U, V, Wf, k, j, i, nz, ihx, ihy, ihz, L);
  const T uxp = U.at(k, j, i), uxm = U.at(k, j, i - 1);
  const T vyp = V.at(k, j, i), vym = V.at(k, j - 1, i);
  const T wzp = k < nz - 1 ? Wf.at(k, j, i) : (T)0, wzm = k > 0 ? Wf.at(k - 1, j, i) : (T)0;
  T tau[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) tau[m] = tin.p[m][id];
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int a = pairs[m][0], b = pairs[m][1];
    const Coarse<T> t{tin.p[m], nx, ny, nz};
    const T t0 = tau[m];
    const T fxp = uxp * h * (t0 + t.at(k, j, i + 1));
    const T fxm = uxm * h * (t.at(k, j, i - 1) + t0);
    const T fyp = vyp * h * (t0 + t.at(k, j + 1, i));
    const T fym = vym * h * (t.at(k, j - 1, i) + t0);
    const T fzp = k < nz - 1 ? wzp * h * (t0 + t.at(k + 1, j, i)) : (T)0;
    const T fzm = k > 0 ? wzm * h * (t.at(k - 1, j, i) + t0) : (T)0;
    T rh = -((fxp - fxm) * ihx + (fyp - fym) * ihy + (fzp - fzm) * ihz);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) rh += L[cc][a] * tau[tidx(cc, b)] + tau[tidx(a, cc)] * L[cc][b];
    rh += (one_m_beta * (L[a][b] + L[b][a]) - t0) * inv_wi;
    tout.p[m][id] = c0 * tn.p[m][id] + c1 * (t0 + dt * rh);
  }
}

}  // namespace

template <typename T>
hipError_t launch_momentum_rhs(const Dims& c, const StepConsts& k, NsIn<T> in, Restricted<T> r,
                               T* ru, T* rv, T* rw, hipStream_t st) {
  const Launch3 L = launch3(c.nx, c.ny, 3 * c.nz);
  hipLaunchKernelGGL(k_momentum_rhs<T>, L.grid, L.block, 0, st, in, r, ru, rv, rw, c.nx, c.ny, c.nz,
                     (T)c.ihx, (T)c.ihy, (T)c.ihz, k);
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
  const Launch3 L = launch3(c.nx, c.ny, c.nz);
  hipLaunchKernelGGL(k_polymer_stage<T>, L.grid, L.block, 0, st, u, v, w, tn, ti, to, c.nx, c.ny, c.nz,
                     (T)c.ihx, (T)c.ihy, (T)c.ihz, (T)k.dt, (T)k.inv_wi, (T)(1.0 - k.beta), (T)c0,
                     (T)c1);
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
