// Coarse-grid (flow) stencils.
//
//   momentum_rhs   -- right-hand side r of the velocity Helmholtz equations of eq. NS36,
//                     (nu_m L - gamma0/dt) u~ = r, for each component at its own faces.
//                     r collects -u_hat/dt (eq. NS35), the conservative central advection of
//                     u*, the diffusive-flux term J.grad(u*)/rho, the split pressure gradient
//                     (1/rho0) grad p^n + (1/rho - 1/rho0) grad p*, the explicit nu_m L u*,
//                     the polymer divergence of the second approach (eq. NS12, drop = polymer
//                     phase), the variable-viscosity stress divergence, the capillary force
//                     G grad(phi) and the body force. 3D grids march up columns (every thread
//                     forms the three components of its cell); 2D grids take one thread per
//                     face. The Oldroyd-B/Giesekus polymer divergence comes from its own
//                     z-marching pass (polymer_div).
//   polymer_stage  -- one stage of the second-order TVD Runge-Kutta update of the polymer
//                     stress (eqs. NS42, NS44) in stress form: the Giesekus law, with
//                     -alpha/(1 - beta) tau.tau (alpha = 0: Oldroyd-B); central or WENO-Z
//                     advection.
//
// Staggering: u[k][j][i] at ((i+1) hx, (j+.5) hy, (k+.5) hz), v at (i+.5, j+1, k+.5),
// w at (i+.5, j+.5, k+1) with w[nz-1] the top wall; centres at (i+.5, j+.5, k+.5).
// Wall rules: no-slip ghost = -adjacent for u, v; w = 0 on the walls; Neumann ghost for
// centred scalars (G, tau). Arithmetic in the storage type T.
#include "coarse.hpp"
#include "weno.hpp"

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
              {in.taun, in.taunm1, R.phi_c, nx, ny, nz, f},
              R,
              in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1,
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

// LDS ring views of the z-marching kernel: per layer a tile of HX x HY points covering the
// block's TX x TY columns with one point of halo below and two above in x and y (one row when
// ny == 1), values stored with their wall rule applied.
template <typename T>
struct RingV {
  const T* sl[3];  // layers k-1, k, k+1
  int k, X0, Y0, ys;
  __device__ __forceinline__ T s(int kk, int jj, int ii) const {
    return sl[kk - k + 1][(jj - Y0 + 1) * ys + (ii - X0 + 1)];
  }
  __device__ __forceinline__ T sd(int kk, int jj, int ii) const { return s(kk, jj, ii); }
  __device__ __forceinline__ T sw(int kk, int jj, int ii) const { return s(kk, jj, ii); }
};
// Weighted polymer stress (1 + phi_c)/2 tau* in LDS: the xz, yz and zz components (read on
// layers k-1 .. k+1) in three-layer rings, the xx, yy and xy components (read on layer k only)
// in one slot each; Neumann clamp applied on load.
template <typename T>
struct RingT {
  const T* r3[3][3];  // [xz, yz, zz][layer k-1, k, k+1]
  const T* r1[3];     // [xx, yy, xy] on layer k
  int k, X0, Y0, ys;
  __device__ __forceinline__ T at(int comp, int kk, int jj, int ii) const {
    const int e = (jj - Y0 + 1) * ys + (ii - X0 + 1);
    switch (comp) {
      case 0: return r1[0][e];
      case 1: return r1[1][e];
      case 3: return r1[2][e];
      case 4: return r3[0][kk - k + 1][e];
      case 5: return r3[1][kk - k + 1][e];
      default: return r3[2][kk - k + 1][e];
    }
  }
};

template <typename T>
struct RingG {
  const T* sl[4];  // layers k-1 .. k+2
  int k, X0, Y0, ys;
  __device__ __forceinline__ T at(int kk, int jj, int ii) const {
    return sl[kk - k + 1][(jj - Y0 + 1) * ys + (ii - X0 + 1)];
  }
  __device__ __forceinline__ T atn(int kk, int jj, int ii) const { return at(kk, jj, ii); }
};

// Halo tile of a z-marching block: TX x TY coarse columns with one point of halo below and two
// above in x and y. Each thread owns at most RP tile points; their in-layer byte offsets (a
// uniform layer base plus a 32-bit lane offset) are computed once.
template <typename T, int RP>
struct HaloTile {
  int HX, HP, tid, nth;
  unsigned off[RP];
  __device__ __forceinline__ HaloTile(int TX, int TY, int X0, int Y0, int nx, int ny) {
    HX = TX + 3;
    HP = HX * (TY + 3);
    tid = threadIdx.y * TX + threadIdx.x;
    nth = TX * TY;
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      const int e = tid + q * nth;
      const int hy = e / HX, hx = e - hy * HX;
      off[q] = e < HP ? (unsigned)(wrap(Y0 - 1 + hy, ny) * nx + wrap(X0 - 1 + hx, nx)) * (unsigned)sizeof(T) : 0u;
    }
  }
  // fn(tile index, byte offset) for every point of this thread
  template <typename F>
  __device__ __forceinline__ void each(F&& fn) const {
#pragma unroll
    for (int q = 0; q < RP; ++q)
      if (tid + q * nth < HP) fn(tid + q * nth, off[q]);
  }
};

// Divergence of the weighted polymer stress (1 + phi_c)/2 tau* at the u, v and w faces,
// z-marching like the momentum kernel: the xz, yz and zz components (read on layers k-1 ..
// k+1) in three-layer LDS rings, the xx, yy and xy components (layer k only) in one slot each,
// Neumann clamp on load. The results go to three arrays shaped like u, v, w (the top-wall w
// face gets zero); the momentum kernel reads them at its own faces.
template <typename T, int RP>
__global__ void __launch_bounds__(kBlock)
    k_polymer_div_zm(NsIn<T> in, const T* __restrict__ phic, int first, int nx, int ny, int nz, int KB,
                     T ihx, T ihy, T ihz) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TX = blockDim.x, TY = blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int X0 = bx * TX, Y0 = by * TY, K0 = bz * KB;
  const HaloTile<T, RP> H(TX, TY, X0, Y0, nx, ny);
  const int HP = H.HP;
  T* sT3 = reinterpret_cast<T*>(smem);  // [xz, yz, zz] x 3 slots
  T* sT1 = sT3 + 9 * HP;                // [xx, yy, xy]
  const size_t layer = (size_t)ny * nx;
  const int i = X0 + threadIdx.x, j = Y0 + threadIdx.y;
  auto load_t = [&](int kk, const int* comps, T* const* dst) {
    const size_t o = min(max(kk, 0), nz - 1) * layer;
    H.each([&](int e, unsigned off) {
      const T w = (T)0.5 * ((T)1 + ld_at(phic + o, off));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T a = ld_at(in.taun[comps[c]] + o, off);
        dst[c][e] = w * (first ? a : (T)2 * a - ld_at(in.taunm1[comps[c]] + o, off));
      }
    });
  };
  const int c3[3] = {4, 5, 2}, c1[3] = {0, 1, 3};
  auto load_t3 = [&](int kk) {
    const int sl = (kk - K0 + 1) % 3;
    T* const dst[3] = {sT3 + (0 * 3 + sl) * HP, sT3 + (1 * 3 + sl) * HP, sT3 + (2 * 3 + sl) * HP};
    load_t(kk, c3, dst);
  };
  auto load_t1 = [&](int kk) {
    T* const dst[3] = {sT1, sT1 + HP, sT1 + 2 * HP};
    load_t(kk, c1, dst);
  };
  load_t3(K0 - 1);
  load_t3(K0);
  const int K1 = min(K0 + KB, nz);  // the last block of a column may march fewer layers
  for (int k = K0; k < K1; ++k) {
    load_t3(k + 1);
    load_t1(k);
    __syncthreads();
    const int t0 = (k - K0) % 3, t1 = (k - K0 + 1) % 3, t2 = (k - K0 + 2) % 3;
    const RingT<T> Tr{{{sT3 + t0 * HP, sT3 + t1 * HP, sT3 + t2 * HP},
                       {sT3 + (3 + t0) * HP, sT3 + (3 + t1) * HP, sT3 + (3 + t2) * HP},
                       {sT3 + (6 + t0) * HP, sT3 + (6 + t1) * HP, sT3 + (6 + t2) * HP}},
                      {sT1, sT1 + HP, sT1 + 2 * HP},
                      k, X0, Y0, H.HX};
    auto tp = [&](int c, int kk, int jj, int ii) { return Tr.at(c, kk, jj, ii); };
    const int id = (k * ny + j) * nx + i;
    in.pol[0][id] = polymer_div_u<T>(tp, k, j, i, ihx, ihy, ihz);
    in.pol[1][id] = polymer_div_v<T>(tp, k, j, i, ihx, ihy, ihz);
    in.pol[2][id] = k == nz - 1 ? (T)0 : polymer_div_w<T>(tp, k, j, i, ihx, ihy, ihz);
    __syncthreads();
  }
}

// Momentum right-hand side, z-marching: a block owns TX x TY coarse columns and KB layers;
// the extrapolated velocities (three-layer rings) and G at centres (four-layer ring, for J)
// live in LDS, every thread forms all three components of its cell from them. The other
// inputs are read once or twice per cell from global memory; VE (Oldroyd-B) adds the face
// divergences of the weighted polymer stress, given by k_polymer_div_zm. Each thread loads at
// most RP points of a halo tile.
template <typename T, bool VE, int RP>
__global__ void __launch_bounds__(kBlock)
    k_momentum_rhs_zm(NsIn<T> in, Restricted<T> R, T* __restrict__ ru, T* __restrict__ rv,
                      T* __restrict__ rw, StepConsts c, int nx, int ny, int nz, int KB, T ihx, T ihy,
                      T ihz) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TX = blockDim.x, TY = blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int X0 = bx * TX, Y0 = by * TY, K0 = bz * KB;
  const HaloTile<T, RP> H(TX, TY, X0, Y0, nx, ny);
  const int HP = H.HP, ys = H.HX;
  T* sU = reinterpret_cast<T*>(smem);
  T* sV = sU + 3 * HP;
  T* sW = sV + 3 * HP;
  T* sG = sW + 3 * HP;
  const int i = X0 + threadIdx.x, j = Y0 + threadIdx.y;
  const int f = c.first;
  const size_t layer = (size_t)ny * nx;
  auto star_at = [&](const T* a, const T* b, unsigned o) {
    return f ? ld_at(a, o) : (T)2 * ld_at(a, o) - ld_at(b, o);
  };
  // extrapolated velocities on layer kk: no-slip ghosts (minus the adjacent layer) for u, v
  // beyond the walls; w is zero on and beyond the walls
  auto load_vel = [&](int kk) {
    const int sl = (kk - K0 + 1) % 3;
    const int kc = min(max(kk, 0), nz - 1);
    const T sg = (kk < 0 || kk >= nz) ? (T)-1 : (T)1;
    const bool wz = kk < 0 || kk >= nz - 1;
    const size_t o = kc * layer;
    const T *ua = in.un + o, *ub = in.unm1 + o, *va = in.vn + o, *vb = in.vnm1 + o;
    const T *wa = in.wn + o, *wb = in.wnm1 + o;
    H.each([&](int e, unsigned off) {
      sU[sl * HP + e] = sg * star_at(ua, ub, off);
      sV[sl * HP + e] = sg * star_at(va, vb, off);
      sW[sl * HP + e] = wz ? (T)0 : star_at(wa, wb, off);
    });
  };
  auto load_g = [&](int kk) {
    const int sl = (kk - K0 + 1) & 3;
    const T* g = R.G_c + min(max(kk, 0), nz - 1) * layer;
    H.each([&](int e, unsigned off) { sG[sl * HP + e] = ld_at(g, off); });
  };
  load_vel(K0 - 1);
  load_vel(K0);
  load_g(K0 - 1);
  load_g(K0);
  load_g(K0 + 1);
  const int K1 = min(K0 + KB, nz);  // the last block of a column may march fewer layers
  for (int k = K0; k < K1; ++k) {
    load_vel(k + 1);
    load_g(k + 2);
    __syncthreads();
    const int v0 = (k - K0) % 3, v1 = (k - K0 + 1) % 3, v2 = (k - K0 + 2) % 3;
    const RingV<T> Ur{{sU + v0 * HP, sU + v1 * HP, sU + v2 * HP}, k, X0, Y0, ys};
    const RingV<T> Vr{{sV + v0 * HP, sV + v1 * HP, sV + v2 * HP}, k, X0, Y0, ys};
    const RingV<T> Wr{{sW + v0 * HP, sW + v1 * HP, sW + v2 * HP}, k, X0, Y0, ys};
    const RingG<T> Gr{{sG + ((k - K0) & 3) * HP, sG + ((k - K0 + 1) & 3) * HP, sG + ((k - K0 + 2) & 3) * HP,
                       sG + ((k - K0 + 3) & 3) * HP},
                      k, X0, Y0, ys};
    const PolPre<T> Pp{{in.pol[0], in.pol[1], in.pol[2]}};
    MomCtxG<T, RingV<T>, RingG<T>, PolPre<T>> m{Ur, Vr, Wr,
                                     {in.pn, in.pnm1, nx, ny, nz, f},
                                     {in.pn, nullptr, nx, ny, nz, 1},
                                     Gr,
                                     {R.phi_c, nx, ny, nz},
                                     {R.mu_c, nx, ny, nz},
                                     {R.mu_xy, nx, ny, nz},
                                     {R.mu_xz, nx, ny},
                                     {R.mu_yz, nx, ny},
                                     Pp,
                                     R,
                                     in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1,
                                     nx, ny, nz, f, VE ? 1 : 0,
                                     ihx, ihy, ihz,
                                     (T)c.inv_dt, (T)c.inv_re, (T)c.inv_rho0, (T)c.nu_m, (T)c.k_sigma, (T)c.c_j};
    auto rhs = [&](const MomTerms<T>& t, T a) -> T {
      return -t.hat * m.inv_dt + t.adv + t.ri * t.jg + t.gpn * m.ir0 + (t.ri - m.ir0) * t.gps + m.nu_m * t.lap -
             m.inv_re * t.ri * t.pol - m.inv_re * t.ri * t.vis - m.k_sigma * t.ri * t.cap - a;
    };
    const int id = (k * ny + j) * nx + i;
    ru[id] = rhs(mom_u(m, k, j, i, id), (T)c.ax);
    rv[id] = rhs(mom_v(m, k, j, i, id), (T)c.ay);
    rw[id] = k == nz - 1 ? (T)0 : rhs(mom_w(m, k, j, i, id), (T)c.az);
    __syncthreads();
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

template <typename T, bool WENO>
__global__ void __launch_bounds__(kBlock)
    k_polymer_stage(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
                    TauSet<T> tn, TauSet<T> tin, TauOut<T> tout, int nx, int ny, int nz, T ihx,
                    T ihy, T ihz, T dt, T inv_wi, T one_m_beta, T gk, T c0, T c1) {
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
  const WenoOffsets<T> wo(k, j, WENO ? i : 0, nx, ny, nz);
  const NbrOffsets<T> no(k, j, i, nx, ny, nz);
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int a = pairs[m][0], b = pairs[m][1];
    const T t0 = tau[m];
    T rh;
    if (WENO) {
      // WENO-Z face values, three cells either way, mirrored beyond the walls
      rh = wo.advection(tin.p[m], uxm, uxp, vym, vyp, wzm, wzp, ihx, ihy, ihz);
    } else {
      const T* q = tin.p[m];
      const T fxp = uxp * h * (t0 + ld_at(q, no.xp));
      const T fxm = uxm * h * (ld_at(q, no.xm) + t0);
      const T fyp = vyp * h * (t0 + ld_at(q, no.yp));
      const T fym = vym * h * (ld_at(q, no.ym) + t0);
      const T fzp = k < nz - 1 ? wzp * h * (t0 + ld_at(q, no.zp)) : (T)0;
      const T fzm = k > 0 ? wzm * h * (ld_at(q, no.zm) + t0) : (T)0;
      rh = -((fxp - fxm) * ihx + (fyp - fym) * ihy + (fzp - fzm) * ihz);
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) rh += L[cc][a] * tau[tidx(cc, b)] + tau[tidx(a, cc)] * L[cc][b];
    rh += (one_m_beta * (L[a][b] + L[b][a]) - t0) * inv_wi;
    // Giesekus: - alpha/(1 - beta) (tau.tau)_ab
    if (gk != (T)0) {
      T tt = 0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) tt += tau[tidx(a, cc)] * tau[tidx(cc, b)];
      rh -= gk * tt;
    }
    tout.p[m][id] = c0 * tn.p[m][id] + c1 * (t0 + dt * rh);
  }
}

}  // namespace

template <typename T>
hipError_t launch_momentum_rhs(const Dims& c, const StepConsts& k, NsIn<T> in, Restricted<T> r,
                               T* ru, T* rv, T* rw, hipStream_t st) {
  if (c.ny == 1) {
    // 2D: too few columns to feed z-marching blocks; one thread per face instead
    const Launch3 L = launch3(c.nx, c.ny, 3 * c.nz);
    hipLaunchKernelGGL(k_momentum_rhs<T>, L.grid, L.block, 0, st, in, r, ru, rv, rw, c.nx, c.ny, c.nz,
                       (T)c.ihx, (T)c.ihy, (T)c.ihz, k);
    return hipGetLastError();
  }
  const int TX = c.nx < 32 ? c.nx : 32;
  const int TY = c.ny < kBlock / TX ? c.ny : kBlock / TX;
  const int cols = (c.nx / TX) * (c.ny / TY);
  const dim3 block(TX, TY);
  // halo points per thread: 2 for tiles of 32 x 4 and up, 4 for the small tiles of small grids
  const int HP = (TX + 3) * (TY + 3);
  const int need = (HP + TX * TY - 1) / (TX * TY);
  if (need > 4) return hipErrorInvalidConfiguration;
  auto go = [&](auto kernel, size_t shm, auto... args) {
    const int KB = march_layers(kernel, TX * TY, shm, cols, c.nz);
    const dim3 grid(c.nx / TX, c.ny / TY, (c.nz + KB - 1) / KB);
    hipLaunchKernelGGL(kernel, grid, block, shm, st, args..., KB, (T)c.ihx, (T)c.ihy, (T)c.ihz);
  };
  if (in.viscoelastic) {
    if (!in.pol[0] || !in.pol[1] || !in.pol[2]) return hipErrorInvalidValue;
    // the face divergences of the weighted polymer stress first (12 LDS tile slots)
    const size_t shp = (size_t)12 * HP * sizeof(T);
    if (need <= 2)
      go(k_polymer_div_zm<T, 2>, shp, in, (const T*)r.phi_c, k.first, c.nx, c.ny, c.nz);
    else
      go(k_polymer_div_zm<T, 4>, shp, in, (const T*)r.phi_c, k.first, c.nx, c.ny, c.nz);
  }
  const size_t shm = (size_t)13 * HP * sizeof(T);
#define DRPF_MOM(VE, RP) go(k_momentum_rhs_zm<T, VE, RP>, shm, in, r, ru, rv, rw, k, c.nx, c.ny, c.nz)
  if (in.viscoelastic) {
    if (need <= 2) DRPF_MOM(true, 2); else DRPF_MOM(true, 4);
  } else {
    if (need <= 2) DRPF_MOM(false, 2); else DRPF_MOM(false, 4);
  }
#undef DRPF_MOM
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
  const T gk = (T)(k.giesekus == 0.0 ? 0.0 : k.giesekus / (1.0 - k.beta));
  if (k.advection == 1)
    hipLaunchKernelGGL((k_polymer_stage<T, true>), L.grid, L.block, 0, st, u, v, w, tn, ti, to, c.nx, c.ny,
                       c.nz, (T)c.ihx, (T)c.ihy, (T)c.ihz, (T)k.dt, (T)k.inv_wi, (T)(1.0 - k.beta), gk, (T)c0,
                       (T)c1);
  else
    hipLaunchKernelGGL((k_polymer_stage<T, false>), L.grid, L.block, 0, st, u, v, w, tn, ti, to, c.nx, c.ny,
                       c.nz, (T)c.ihx, (T)c.ihy, (T)c.ihz, (T)k.dt, (T)k.inv_wi, (T)(1.0 - k.beta), gk, (T)c0,
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
