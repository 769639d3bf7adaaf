// Coarse-grid accessors and the terms of the momentum right-hand side (eq. NS36), shared by
// the forward momentum kernel and its adjoint. Staggering: u[k][j][i] at ((i+1) hx,
// (j+.5) hy, (k+.5) hz), v at (i+.5, j+1, k+.5), w at (i+.5, j+.5, k+1) with w[nz-1] the top
// wall; centres at (i+.5, j+.5, k+.5). Wall rules: no-slip ghost = 2 u_w - adjacent for u, v
// (eq. NS13; -adjacent for walls at rest); w = 0 on the walls; Neumann ghost for centred
// scalars (G, tau).
#pragma once

#include "kernels.hpp"

namespace drpf {

template <typename T>
struct Field {
  const T* a;
  const T* b;   // level n-1 (extrapolation) or null
  int nx, ny, nz, first;
  T wb = 0, wt = 0;  // wall values at z = 0 and z = lz (no-slip components)
  // 32-bit element indices: every supported grid has fewer than 2^31 cells per array
  __device__ __forceinline__ int idx(int k, int j, int i) const {
    return (k * ny + wrap(j, ny)) * nx + wrap(i, nx);
  }
  // extrapolated value (u* = 2 u^n - u^{n-1}, or u^n on the first step), in-range k
  __device__ __forceinline__ T s(int k, int j, int i) const {
    const int id = idx(k, j, i);
    return (first || b == nullptr) ? a[id] : (T)2 * a[id] - b[id];
  }
  __device__ __forceinline__ T n(int k, int j, int i) const { return a[idx(k, j, i)]; }
  // cell-centred-in-z velocity with no-slip ghosts (2 wall - adjacent)
  __device__ __forceinline__ T sd(int k, int j, int i) const {
    if (k < 0) return (T)2 * wb - s(0, j, i);
    if (k >= nz) return (T)2 * wt - s(nz - 1, j, i);
    return s(k, j, i);
  }
  // z-face velocity: index -1 is the bottom wall, nz-1 the top wall, beyond 0
  __device__ __forceinline__ T sw(int k, int j, int i) const {
    if (k < 0 || k >= nz - 1) return (T)0;
    return s(k, j, i);
  }
  // centred scalar with Neumann ghosts
  __device__ __forceinline__ T sn(int k, int j, int i) const { return s(min(max(k, 0), nz - 1), j, i); }
};

template <typename T>
struct Coarse {
  const T* a;
  int nx, ny, nz;
  __device__ __forceinline__ T at(int k, int j, int i) const {
    return a[(k * ny + wrap(j, ny)) * nx + wrap(i, nx)];
  }
  __device__ __forceinline__ T atn(int k, int j, int i) const { return at(min(max(k, 0), nz - 1), j, i); }
};

// z-edge arrays (nz + 1 layers): layer m is the edge at z = m hz
template <typename T>
struct ZEdge {
  const T* a;
  int nx, ny;
  __device__ __forceinline__ T at(int m, int j, int i) const {
    return a[(m * ny + wrap(j, ny)) * nx + wrap(i, nx)];
  }
};

// The separately evaluated terms of one velocity component's right-hand side at one face.
// The right-hand side is
//   -hat/dt + adv + ri jg + gpn/rho0 + (ri - 1/rho0) gps + nu_m lap
//   - (1/Re) ri pol - (1/Re) ri vis - k_sigma ri cap - a_ext.
template <typename T>
struct MomTerms {
  T hat, adv, jg, gpn, gps, lap, pol, vis, cap, ri;
};

// Polymer stress weighted by the polymer fraction, (1 + phi_c)/2 tau*, at centres with Neumann
// ghosts, read from global memory.
template <typename T>
struct TauW {
  static constexpr bool pre = false;
  const T* const* taun;
  const T* const* taunm1;
  const T* phic;
  int nx, ny, nz, first;
  __device__ __forceinline__ T at(int comp, int k, int j, int i) const {
    const int kc = min(max(k, 0), nz - 1);
    const int id = (kc * ny + wrap(j, ny)) * nx + wrap(i, nx);
    const T a = taun[comp][id];
    const T ts = first ? a : (T)2 * a - taunm1[comp][id];
    return (T)0.5 * ((T)1 + phic[id]) * ts;
  }
};

// Divergence of the weighted polymer stress at the u, v and w faces of cell (k, j, i), from an
// accessor tp(comp, k, j, i) of the weighted stress at centres (comp: xx, yy, zz, xy, xz, yz):
// the normal component by a face difference, the shear components averaged to the edges
// first.
template <typename T, typename TP>
__device__ __forceinline__ T polymer_div_u(const TP& tp, int k, int j, int i, T ihx, T ihy, T ihz) {
  const T q = (T)0.25;
  auto txy = [&](int jj) { return q * (tp(3, k, jj, i) + tp(3, k, jj, i + 1) + tp(3, k, jj + 1, i) + tp(3, k, jj + 1, i + 1)); };
  auto txz = [&](int kk) { return q * (tp(4, kk, j, i) + tp(4, kk, j, i + 1) + tp(4, kk + 1, j, i) + tp(4, kk + 1, j, i + 1)); };
  return (tp(0, k, j, i + 1) - tp(0, k, j, i)) * ihx + (txy(j) - txy(j - 1)) * ihy + (txz(k) - txz(k - 1)) * ihz;
}
template <typename T, typename TP>
__device__ __forceinline__ T polymer_div_v(const TP& tp, int k, int j, int i, T ihx, T ihy, T ihz) {
  const T q = (T)0.25;
  auto txy = [&](int ii) { return q * (tp(3, k, j, ii) + tp(3, k, j, ii + 1) + tp(3, k, j + 1, ii) + tp(3, k, j + 1, ii + 1)); };
  auto tyz = [&](int kk) { return q * (tp(5, kk, j, i) + tp(5, kk, j + 1, i) + tp(5, kk + 1, j, i) + tp(5, kk + 1, j + 1, i)); };
  return (txy(i) - txy(i - 1)) * ihx + (tp(1, k, j + 1, i) - tp(1, k, j, i)) * ihy + (tyz(k) - tyz(k - 1)) * ihz;
}
template <typename T, typename TP>
__device__ __forceinline__ T polymer_div_w(const TP& tp, int k, int j, int i, T ihx, T ihy, T ihz) {
  const T q = (T)0.25;
  auto txz = [&](int ii) { return q * (tp(4, k, j, ii) + tp(4, k, j, ii + 1) + tp(4, k + 1, j, ii) + tp(4, k + 1, j, ii + 1)); };
  auto tyz = [&](int jj) { return q * (tp(5, k, jj, i) + tp(5, k, jj + 1, i) + tp(5, k + 1, jj, i) + tp(5, k + 1, jj + 1, i)); };
  return (txz(i) - txz(i - 1)) * ihx + (tyz(j) - tyz(j - 1)) * ihy + (tp(2, k + 1, j, i) - tp(2, k, j, i)) * ihz;
}

// The three face divergences precomputed by a separate pass (arrays shaped like u, v, w).
template <typename T>
struct PolPre {
  static constexpr bool pre = true;
  const T* p[3];
};

// Inputs of the momentum right-hand side. VA reads the extrapolated velocities (methods s, sd,
// sw as in Field), GA the restricted chemical potential at centres (at, atn as in Coarse) and
// TA the weighted polymer stress (at as in TauW, from global memory or LDS rings; or PolPre,
// whose pre flag says that the face divergences are given); PA the pressure (s, n as in
// Field), CA phi_c and mu_c (at as in Coarse), EA the z-edge viscosities (at as in ZEdge),
// from memory or through a register cache of the caller's own column; HA the level n-1
// velocities at the face (PrevMem, or values the caller holds).
// The level n-1 velocities at the face being formed (the hat of eq. NS31), read from memory
template <typename T>
struct PrevMem {
  template <typename C>
  __device__ __forceinline__ T at(const C& m, int comp, int id) const {
    return (comp == 0 ? m.unm1 : comp == 1 ? m.vnm1 : m.wnm1)[id];
  }
};

template <typename T, typename VA, typename GA, typename TA = TauW<T>, typename PA = Field<T>,
          typename CA = Coarse<T>, typename EA = ZEdge<T>, typename HA = PrevMem<T>>
struct MomCtxG {
  using value_type = T;
  VA U, V, W;
  PA P, Pn;  // P: s (extrapolated pressure), Pn: n (pressure at level n)
  GA Gc;
  CA phic, muc;
  Coarse<T> muxy;
  EA muxz, muyz;
  TA Tw;
  Restricted<T> R;
  const T *un, *unm1, *vn, *vnm1, *wn, *wnm1;  // levels n, n-1 (n-1 for the hat of eq. NS31)
  int nx, ny, nz, first, ve;
  T ihx, ihy, ihz;
  T inv_dt, inv_re, ir0, nu_m, k_sigma, c_j;
  HA prev = {};  // level n-1 velocity at the face (memory, or the caller's registers)
  // hat of eq. NS31 at an in-range face from the extrapolated value there: 2 u^n - u^{n-1}/2 =
  // u* + u^{n-1}/2 with u* = 2 u^n - u^{n-1}; u^n (= u*) on the first step
  __device__ __forceinline__ T hat(T star, int comp, int id) const {
    return first ? star : star + (T)0.5 * prev.at(*this, comp, id);
  }
  // J = -c_j grad G at a centre: 2h central differences, Neumann in z
  __device__ __forceinline__ void Jc(int k, int j, int i, T* J) const {
    const T h = (T)0.5;
    J[0] = -c_j * (Gc.at(k, j, i + 1) - Gc.at(k, j, i - 1)) * h * ihx;
    J[1] = -c_j * (Gc.at(k, j + 1, i) - Gc.at(k, j - 1, i)) * h * ihy;
    J[2] = -c_j * (Gc.atn(k + 1, j, i) - Gc.atn(k - 1, j, i)) * h * ihz;
  }
  // polymer weight (1 + phi_c)/2 tau*, Neumann ghosts
  __device__ __forceinline__ T Tp(int comp, int k, int j, int i) const { return Tw.at(comp, k, j, i); }
};

template <typename T>
using MomCtx = MomCtxG<T, Field<T>, Coarse<T>>;

template <typename C>
__device__ __forceinline__ MomTerms<typename C::value_type> mom_u(const C& m, int k, int j, int i, int id) {
  using T = typename C::value_type;
  const auto& U = m.U;
  const auto& V = m.V;
  const auto& W = m.W;
  const T h = (T)0.5, ihx = m.ihx, ihy = m.ihy, ihz = m.ihz;
  const T u0 = U.s(k, j, i);
  const T uxp = U.s(k, j, i + 1), uxm = U.s(k, j, i - 1);
  const T uyp = U.s(k, j + 1, i), uym = U.s(k, j - 1, i);
  const T uzp = U.sd(k + 1, j, i), uzm = U.sd(k - 1, j, i);
  // advection
  const T ucr = h * (u0 + uxp), ucl = h * (uxm + u0);
  T adv = (ucr * ucr - ucl * ucl) * ihx;
  const T v00 = V.s(k, j, i), v01 = V.s(k, j, i + 1), vm0 = V.s(k, j - 1, i), vm1 = V.s(k, j - 1, i + 1);
  adv += (h * (v00 + v01) * h * (u0 + uyp) - h * (vm0 + vm1) * h * (uym + u0)) * ihy;
  const T w00 = W.sw(k, j, i), w01 = W.sw(k, j, i + 1), wm0 = W.sw(k - 1, j, i), wm1 = W.sw(k - 1, j, i + 1);
  adv += (h * (w00 + w01) * h * (u0 + uzp) - h * (wm0 + wm1) * h * (uzm + u0)) * ihz;
  // J . grad u*
  T Ja[3], Jb[3];
  m.Jc(k, j, i, Ja);
  m.Jc(k, j, i + 1, Jb);
  const T jgu = h * (Ja[0] + Jb[0]) * (uxp - uxm) * h * ihx + h * (Ja[1] + Jb[1]) * (uyp - uym) * h * ihy +
                h * (Ja[2] + Jb[2]) * (uzp - uzm) * h * ihz;
  // viscous stress divergence
  T vis = ((T)2 * m.muc.at(k, j, i + 1) * (uxp - u0) * ihx - (T)2 * m.muc.at(k, j, i) * (u0 - uxm) * ihx) * ihx;
  const T sxyp = m.muxy.at(k, j, i) * ((uyp - u0) * ihy + (v01 - v00) * ihx);
  const T sxym = m.muxy.at(k, j - 1, i) * ((u0 - uym) * ihy + (vm1 - vm0) * ihx);
  vis += (sxyp - sxym) * ihy;
  const T sxzp = m.muxz.at(k + 1, j, i) * ((uzp - u0) * ihz + (w01 - w00) * ihx);
  const T sxzm = m.muxz.at(k, j, i) * ((u0 - uzm) * ihz + (wm1 - wm0) * ihx);
  vis += (sxzp - sxzm) * ihz;
  // polymer divergence
  T pol = 0;
  if (m.ve) {
    if constexpr (decltype(m.Tw)::pre)
      pol = m.Tw.p[0][id];
    else
      pol = polymer_div_u<T>([&](int c, int kk, int jj, int ii) { return m.Tp(c, kk, jj, ii); }, k, j, i, ihx, ihy, ihz);
  }
  const T ri = m.R.ri_x[id];
  const T gpn = (m.Pn.n(k, j, i + 1) - m.Pn.n(k, j, i)) * ihx;
  const T gps = (m.P.s(k, j, i + 1) - m.P.s(k, j, i)) * ihx;
  const T cap = m.R.G_x[id] * (m.phic.at(k, j, i + 1) - m.phic.at(k, j, i)) * ihx;
  const T lap = (uxp - 2 * u0 + uxm) * ihx * ihx + (uyp - 2 * u0 + uym) * ihy * ihy + (uzp - 2 * u0 + uzm) * ihz * ihz;
  return MomTerms<T>{m.hat(u0, 0, id), adv, jgu, gpn, gps, lap, pol, vis, cap, ri};
}

template <typename C>
__device__ __forceinline__ MomTerms<typename C::value_type> mom_v(const C& m, int k, int j, int i, int id) {
  using T = typename C::value_type;
  const auto& U = m.U;
  const auto& V = m.V;
  const auto& W = m.W;
  const T h = (T)0.5, ihx = m.ihx, ihy = m.ihy, ihz = m.ihz;
  const T v0 = V.s(k, j, i);
  const T vxp = V.s(k, j, i + 1), vxm = V.s(k, j, i - 1);
  const T vyp = V.s(k, j + 1, i), vym = V.s(k, j - 1, i);
  const T vzp = V.sd(k + 1, j, i), vzm = V.sd(k - 1, j, i);
  const T vcu = h * (v0 + vyp), vcl = h * (vym + v0);
  T adv = (vcu * vcu - vcl * vcl) * ihy;
  const T u00 = U.s(k, j, i), u10 = U.s(k, j + 1, i), u0m = U.s(k, j, i - 1), u1m = U.s(k, j + 1, i - 1);
  adv += (h * (u00 + u10) * h * (v0 + vxp) - h * (u0m + u1m) * h * (vxm + v0)) * ihx;
  const T w00 = W.sw(k, j, i), w10 = W.sw(k, j + 1, i), wm0 = W.sw(k - 1, j, i), wm1 = W.sw(k - 1, j + 1, i);
  adv += (h * (w00 + w10) * h * (v0 + vzp) - h * (wm0 + wm1) * h * (vzm + v0)) * ihz;
  T Ja[3], Jb[3];
  m.Jc(k, j, i, Ja);
  m.Jc(k, j + 1, i, Jb);
  const T jgv = h * (Ja[0] + Jb[0]) * (vxp - vxm) * h * ihx + h * (Ja[1] + Jb[1]) * (vyp - vym) * h * ihy +
                h * (Ja[2] + Jb[2]) * (vzp - vzm) * h * ihz;
  T vis = ((T)2 * m.muc.at(k, j + 1, i) * (vyp - v0) * ihy - (T)2 * m.muc.at(k, j, i) * (v0 - vym) * ihy) * ihy;
  const T sxyp = m.muxy.at(k, j, i) * ((u10 - u00) * ihy + (vxp - v0) * ihx);
  const T sxym = m.muxy.at(k, j, i - 1) * ((u1m - u0m) * ihy + (v0 - vxm) * ihx);
  vis += (sxyp - sxym) * ihx;
  const T syzp = m.muyz.at(k + 1, j, i) * ((vzp - v0) * ihz + (w10 - w00) * ihy);
  const T syzm = m.muyz.at(k, j, i) * ((v0 - vzm) * ihz + (wm1 - wm0) * ihy);
  vis += (syzp - syzm) * ihz;
  T pol = 0;
  if (m.ve) {
    if constexpr (decltype(m.Tw)::pre)
      pol = m.Tw.p[1][id];
    else
      pol = polymer_div_v<T>([&](int c, int kk, int jj, int ii) { return m.Tp(c, kk, jj, ii); }, k, j, i, ihx, ihy, ihz);
  }
  const T ri = m.R.ri_y[id];
  const T gpn = (m.Pn.n(k, j + 1, i) - m.Pn.n(k, j, i)) * ihy;
  const T gps = (m.P.s(k, j + 1, i) - m.P.s(k, j, i)) * ihy;
  const T cap = m.R.G_y[id] * (m.phic.at(k, j + 1, i) - m.phic.at(k, j, i)) * ihy;
  const T lap = (vxp - 2 * v0 + vxm) * ihx * ihx + (vyp - 2 * v0 + vym) * ihy * ihy + (vzp - 2 * v0 + vzm) * ihz * ihz;
  return MomTerms<T>{m.hat(v0, 1, id), adv, jgv, gpn, gps, lap, pol, vis, cap, ri};
}

template <typename C>
__device__ __forceinline__ MomTerms<typename C::value_type> mom_w(const C& m, int k, int j, int i, int id) {
  using T = typename C::value_type;
  const auto& U = m.U;
  const auto& V = m.V;
  const auto& W = m.W;
  const T h = (T)0.5, ihx = m.ihx, ihy = m.ihy, ihz = m.ihz;
  const T w0 = W.sw(k, j, i);
  const T wxp = W.sw(k, j, i + 1), wxm = W.sw(k, j, i - 1);
  const T wyp = W.sw(k, j + 1, i), wym = W.sw(k, j - 1, i);
  const T wzp = W.sw(k + 1, j, i), wzm = W.sw(k - 1, j, i);
  const T wcu = h * (w0 + wzp), wcl = h * (wzm + w0);
  T adv = (wcu * wcu - wcl * wcl) * ihz;
  const T u00 = U.s(k, j, i), u10 = U.s(k + 1, j, i), u0m = U.s(k, j, i - 1), u1m = U.s(k + 1, j, i - 1);
  adv += (h * (u00 + u10) * h * (w0 + wxp) - h * (u0m + u1m) * h * (wxm + w0)) * ihx;
  const T v00 = V.s(k, j, i), v10 = V.s(k + 1, j, i), v0m = V.s(k, j - 1, i), v1m = V.s(k + 1, j - 1, i);
  adv += (h * (v00 + v10) * h * (w0 + wyp) - h * (v0m + v1m) * h * (wym + w0)) * ihy;
  T Ja[3], Jb[3];
  m.Jc(k, j, i, Ja);
  m.Jc(k + 1, j, i, Jb);
  const T jgw = h * (Ja[0] + Jb[0]) * (wxp - wxm) * h * ihx + h * (Ja[1] + Jb[1]) * (wyp - wym) * h * ihy +
                h * (Ja[2] + Jb[2]) * (wzp - wzm) * h * ihz;
  T vis = ((T)2 * m.muc.at(k + 1, j, i) * (wzp - w0) * ihz - (T)2 * m.muc.at(k, j, i) * (w0 - wzm) * ihz) * ihz;
  const T sxzp = m.muxz.at(k + 1, j, i) * ((wxp - w0) * ihx + (u10 - u00) * ihz);
  const T sxzm = m.muxz.at(k + 1, j, i - 1) * ((w0 - wxm) * ihx + (u1m - u0m) * ihz);
  vis += (sxzp - sxzm) * ihx;
  const T syzp = m.muyz.at(k + 1, j, i) * ((wyp - w0) * ihy + (v10 - v00) * ihz);
  const T syzm = m.muyz.at(k + 1, j - 1, i) * ((w0 - wym) * ihy + (v1m - v0m) * ihz);
  vis += (syzp - syzm) * ihy;
  T pol = 0;
  if (m.ve) {
    if constexpr (decltype(m.Tw)::pre)
      pol = m.Tw.p[2][id];
    else
      pol = polymer_div_w<T>([&](int c, int kk, int jj, int ii) { return m.Tp(c, kk, jj, ii); }, k, j, i, ihx, ihy, ihz);
  }
  const T ri = m.R.ri_z[id];
  const T gpn = (m.Pn.n(k + 1, j, i) - m.Pn.n(k, j, i)) * ihz;
  const T gps = (m.P.s(k + 1, j, i) - m.P.s(k, j, i)) * ihz;
  const T cap = m.R.G_z[id] * (m.phic.at(k + 1, j, i) - m.phic.at(k, j, i)) * ihz;
  const T lap = (wxp - 2 * w0 + wxm) * ihx * ihx + (wyp - 2 * w0 + wym) * ihy * ihy + (wzp - 2 * w0 + wzm) * ihz * ihz;
  return MomTerms<T>{m.hat(w0, 2, id), adv, jgw, gpn, gps, lap, pol, vis, cap, ri};
}


// tau component index of the pair (a, b): xx, yy, zz, xy, xz, yz
__device__ __forceinline__ int tidx(int a, int b) {
  if (a == b) return a;
  return 2 + a + b;  // 1: xy, 2: xz, 3: yz
}

// Tangential wall velocities (eq. NS13): u and v at z = 0 (ub, vb) and z = lz (ut, vt).
template <typename T>
struct Walls {
  T ub = 0, ut = 0, vb = 0, vt = 0;
};

template <typename T>
__host__ __device__ inline Walls<T> walls_of(const StepConsts& k) {
  Walls<T> w;
  w.ub = (T)k.uwb[0];
  w.ut = (T)k.uwt[0];
  w.vb = (T)k.uwb[1];
  w.vt = (T)k.uwt[1];
  return w;
}

// Velocity gradient at the centre (k, j, i) as L[a][b] = d u_b / d x_a: diagonal entries from
// the compact face difference, off-diagonal ones from the 2h central difference of the
// cell-centred velocity, whose wall ghost is twice the wall velocity minus the adjacent value.
// A reads the face velocities by at(k, j, i) (Coarse, or an LDS view).
template <typename T, typename A>
__device__ __forceinline__ void velocity_gradient(const A& U, const A& V, const A& W, int k, int j,
                                                  int i, int nz, T ihx, T ihy, T ihz, T L[3][3],
                                                  const Walls<T>& wl = Walls<T>{}) {
  const T h = (T)0.5;
  auto wv = [&](int kk, int jj, int ii) -> T { return (kk < 0 || kk >= nz - 1) ? (T)0 : W.at(kk, jj, ii); };
  auto uc = [&](int kk, int jj, int ii) -> T {
    const int kc = min(max(kk, 0), nz - 1);
    const T val = h * (U.at(kc, jj, ii) + U.at(kc, jj, ii - 1));
    return kk == kc ? val : (T)2 * (kk < kc ? wl.ub : wl.ut) - val;
  };
  auto vc = [&](int kk, int jj, int ii) -> T {
    const int kc = min(max(kk, 0), nz - 1);
    const T val = h * (V.at(kc, jj, ii) + V.at(kc, jj - 1, ii));
    return kk == kc ? val : (T)2 * (kk < kc ? wl.vb : wl.vt) - val;
  };
  auto wc = [&](int kk, int jj, int ii) -> T { return h * (wv(kk, jj, ii) + wv(kk - 1, jj, ii)); };
  L[0][0] = (U.at(k, j, i) - U.at(k, j, i - 1)) * ihx;
  L[1][1] = (V.at(k, j, i) - V.at(k, j - 1, i)) * ihy;
  L[2][2] = (wv(k, j, i) - wv(k - 1, j, i)) * ihz;
  L[0][1] = (vc(k, j, i + 1) - vc(k, j, i - 1)) * h * ihx;
  L[0][2] = (wc(k, j, i + 1) - wc(k, j, i - 1)) * h * ihx;
  L[1][0] = (uc(k, j + 1, i) - uc(k, j - 1, i)) * h * ihy;
  L[1][2] = (wc(k, j + 1, i) - wc(k, j - 1, i)) * h * ihy;
  L[2][0] = (uc(k + 1, j, i) - uc(k - 1, j, i)) * h * ihz;
  L[2][1] = (vc(k + 1, j, i) - vc(k - 1, j, i)) * h * ihz;
}

}  // namespace drpf
