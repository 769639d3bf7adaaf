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
// Wall rules: no-slip ghost = 2 u_w - adjacent for u, v (eq. NS13, u = u_w); w = 0 on the
// walls; Neumann ghost for centred scalars (G, tau). Arithmetic in the storage type T.
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
  MomCtx<T> m{{in.un, in.unm1, nx, ny, nz, f, (T)c.uwb[0], (T)c.uwt[0]},
              {in.vn, in.vnm1, nx, ny, nz, f, (T)c.uwb[1], (T)c.uwt[1]},
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

// Register cache of a z-marching thread's own column (j0, i0): the values on layers k0 and
// k0 + 1 (the latter loaded one step ahead and carried to the next layer as its k0 value);
// every other point is read from memory. The comparisons fold away once inlined, since the
// caller passes its own indices.
template <typename T>
struct PCol {  // pressure: extrapolated (s) and level-n (n) values
  Field<T> g;
  int k0, j0, i0;
  T s0, s1, n0, n1;
  __device__ __forceinline__ T s(int k, int j, int i) const {
    if (j == j0 && i == i0) {
      if (k == k0) return s0;
      if (k == k0 + 1) return s1;
    }
    return g.s(k, j, i);
  }
  __device__ __forceinline__ T n(int k, int j, int i) const {
    if (j == j0 && i == i0) {
      if (k == k0) return n0;
      if (k == k0 + 1) return n1;
    }
    return g.n(k, j, i);
  }
};
template <typename T, typename A>
struct ACol {  // a Coarse or ZEdge array
  A g;
  int k0, j0, i0;
  T c0, c1;
  __device__ __forceinline__ T at(int k, int j, int i) const {
    if (j == j0 && i == i0) {
      if (k == k0) return c0;
      if (k == k0 + 1) return c1;
    }
    return g.at(k, j, i);
  }
};

// Halo tile of a z-marching block: TX x TY coarse columns with one point of halo below and two
// above in x and y. Each thread owns at most RP tile points; their in-layer byte offsets (a
// uniform layer base plus a 32-bit lane offset) are computed once. OWN: the points of
// own_first_point (a thread's first point is its own column, so that it also holds its own
// cell's loaded values); otherwise point q of thread t is tile index t + q TX TY.
template <typename T, int RP, bool OWN = false>
struct HaloTile {
  int HX, HP, tid, nth;
  int e[RP];
  unsigned off[RP];
  __device__ __forceinline__ HaloTile(int TX, int TY, int X0, int Y0, int nx, int ny) {
    HX = TX + 3;
    HP = HX * (TY + 3);
    tid = threadIdx.y * TX + threadIdx.x;
    nth = TX * TY;
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      int hy = 0, hx = 0;
      if (!OWN) {
        const int eq = tid + q * nth;
        hy = eq / HX;
        hx = eq - hy * HX;
      } else {
        e[q] = own_first_point<1, 2>(TX, TY, tid, q, hy, hx) ? hy * HX + hx : HP;  // HP: no point
      }
      off[q] = pt(q) < HP ? (unsigned)(wrap(Y0 - 1 + hy, ny) * nx + wrap(X0 - 1 + hx, nx)) * (unsigned)sizeof(T) : 0u;
    }
  }
  // tile index of point q (HP or more: no point)
  __device__ __forceinline__ int pt(int q) const { return OWN ? e[q] : tid + q * nth; }
  // fn(tile index, byte offset) for every point of this thread
  template <typename F>
  __device__ __forceinline__ void each(F&& fn) const {
#pragma unroll
    for (int q = 0; q < RP; ++q)
      if (pt(q) < HP) fn(pt(q), off[q]);
  }
  // fn(q, tile index, byte offset): point q = 0 is the thread's own column when OWN
  template <typename F>
  __device__ __forceinline__ void each_q(F&& fn) const {
#pragma unroll
    for (int q = 0; q < RP; ++q)
      if (pt(q) < HP) fn(q, pt(q), off[q]);
  }
};

// Level n-1 velocities of the caller's own face, held in registers
template <typename T>
struct PrevOwn {
  T v[3];
  template <typename C>
  __device__ __forceinline__ T at(const C&, int comp, int) const {
    return v[comp];
  }
};

// Divergence of the weighted polymer stress (1 + phi_c)/2 tau* at the u, v and w faces,
// z-marching like the momentum kernel: the xz, yz and zz components (read on layers k-1 ..
// k+1) in three-layer LDS rings, the xx, yy and xy components (layer k only) in one slot each,
// Neumann clamp on load. The results go to three arrays shaped like u, v, w (the top-wall w
// face gets zero); the momentum kernel reads them at its own faces.
template <typename T, int RP, int TXC = 0, int NT = kBlock>
__global__ void __launch_bounds__(NT)
    k_polymer_div_zm(NsIn<T> in, const T* __restrict__ phic, int first, int nx, int ny, int nz, int KB,
                     T ihx, T ihy, T ihz) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TX = TXC > 0 ? TXC : (int)blockDim.x, TY = TXC > 0 ? NT / TXC : (int)blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int X0 = bx * TX, Y0 = by * TY, K0 = bz * KB;
  const HaloTile<T, RP, true> H(TX, TY, X0, Y0, nx, ny);
  const int HP = H.HP;
  T* sT3 = reinterpret_cast<T*>(smem);  // [xz, yz, zz] x 3 slots (layers k-1 .. k+1)
  T* sT1 = sT3 + 9 * HP;                // [xx, yy, xy] x 2 slots (layers of either parity)
  const size_t layer = (size_t)ny * nx;
  const int i = X0 + threadIdx.x, j = Y0 + threadIdx.y;
  // raw values of one layer at this thread's tile points (phi_c, tau^n and tau^(n-1) of the six
  // components), loaded one layer ahead of their use
  T rw[RP], ra[RP][6], rb[RP][6];
  auto fetch = [&](int kk) {
    const size_t o = min(max(kk, 0), nz - 1) * layer;
    H.each_q([&](int q, int, unsigned off) {
      rw[q] = ld_at(phic + o, off);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        ra[q][c] = ld_at(in.taun[c] + o, off);
        rb[q][c] = first ? (T)0 : ld_at(in.taunm1[c] + o, off);
      }
    });
  };
  // the weighted stress of the fetched layer kk into its slots: xz, yz, zz into the ring, xx,
  // yy, xy into the slot of kk's parity
  auto put = [&](int kk) {
    const int s3 = (kk - K0 + 1) % 3, s1 = (kk - K0 + 1) & 1;
    H.each_q([&](int q, int e, unsigned) {
      const T w = (T)0.5 * ((T)1 + rw[q]);
      T v[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = w * (first ? ra[q][c] : (T)2 * ra[q][c] - rb[q][c]);
      sT3[(0 * 3 + s3) * HP + e] = v[4];
      sT3[(1 * 3 + s3) * HP + e] = v[5];
      sT3[(2 * 3 + s3) * HP + e] = v[2];
      sT1[(0 * 2 + s1) * HP + e] = v[0];
      sT1[(1 * 2 + s1) * HP + e] = v[1];
      sT1[(2 * 2 + s1) * HP + e] = v[3];
    });
  };
  fetch(K0 - 1);
  put(K0 - 1);
  fetch(K0);
  put(K0);
  fetch(K0 + 1);
  const int K1 = min(K0 + KB, nz);  // the last block of a column may march fewer layers
  for (int k = K0; k < K1; ++k) {
    put(k + 1);
    __syncthreads();
    if (k + 2 <= K1) fetch(k + 2);  // in flight while layer k is formed
    const int t0 = (k - K0) % 3, t1 = (k - K0 + 1) % 3, t2 = (k - K0 + 2) % 3, p1 = (k - K0 + 1) & 1;
    const RingT<T> Tr{{{sT3 + t0 * HP, sT3 + t1 * HP, sT3 + t2 * HP},
                       {sT3 + (3 + t0) * HP, sT3 + (3 + t1) * HP, sT3 + (3 + t2) * HP},
                       {sT3 + (6 + t0) * HP, sT3 + (6 + t1) * HP, sT3 + (6 + t2) * HP}},
                      {sT1 + p1 * HP, sT1 + (2 + p1) * HP, sT1 + (4 + p1) * HP},
                      k, X0, Y0, H.HX};
    auto tp = [&](int c, int kk, int jj, int ii) { return Tr.at(c, kk, jj, ii); };
    const int id = (k * ny + j) * nx + i;
    st_nt(in.pol[0] + id, polymer_div_u<T>(tp, k, j, i, ihx, ihy, ihz));
    st_nt(in.pol[1] + id, polymer_div_v<T>(tp, k, j, i, ihx, ihy, ihz));
    st_nt(in.pol[2] + id, k == nz - 1 ? (T)0 : polymer_div_w<T>(tp, k, j, i, ihx, ihy, ihz));
    __syncthreads();
  }
}

// Momentum right-hand side, z-marching: a block owns TX x TY coarse columns and KB layers;
// the extrapolated velocities (three-layer rings) and G at centres (four-layer ring, for J)
// live in LDS, every thread forms all three components of its cell from them. The other
// inputs are read once or twice per cell from global memory; VE (Oldroyd-B) adds the face
// divergences of the weighted polymer stress, given by k_polymer_div_zm. Each thread loads at
// most RP points of a halo tile. (Five wavefronts per SIMD instead of four spill eight FP32
// registers: no faster, and the reloads add 0.3 GB of HBM reads per launch at 256 x 256 x 128.)
template <typename T, bool VE, int RP, int TXC = 0, int NT = kBlock>
__global__ void __launch_bounds__(NT)
    k_momentum_rhs_zm(NsIn<T> in, Restricted<T> R, T* __restrict__ ru, T* __restrict__ rv,
                      T* __restrict__ rw, StepConsts c, int nx, int ny, int nz, int KB, T ihx, T ihy,
                      T ihz) {
  extern __shared__ __align__(16) unsigned char smem[];
  // TXC > 0: the block shape TXC x (256 / TXC) known at compile time (ring neighbours at
  // immediate offsets)
  const int TX = TXC > 0 ? TXC : (int)blockDim.x, TY = TXC > 0 ? NT / TXC : (int)blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int X0 = bx * TX, Y0 = by * TY, K0 = bz * KB;
  const HaloTile<T, RP, true> H(TX, TY, X0, Y0, nx, ny);
  const int HP = H.HP, ys = H.HX;
  T* sU = reinterpret_cast<T*>(smem);
  T* sV = sU + 3 * HP;
  T* sW = sV + 3 * HP;
  T* sG = sW + 3 * HP;
  const int i = X0 + threadIdx.x, j = Y0 + threadIdx.y;
  const int f = c.first;
  const size_t layer = (size_t)ny * nx;
  // own level n-1 velocities of the layer last put into the ring (see put_vel)
  T prev_next[3] = {(T)0, (T)0, (T)0};
  // With two points per thread and the block shape at compile time, the raw values of the next
  // layer are loaded into registers one layer ahead of their LDS slots, so that the loads are in
  // flight while the current layer is formed. PF (FP32): u^n, u^{n-1}, v^n, v^{n-1}, w^n,
  // w^{n-1} and G, 14 registers, within the 128 that four wavefronts per SIMD allow. PG: G,
  // also in FP64 (4 registers, 164 of the 168 that three wavefronts allow; the velocities would
  // need 24 more, so FP64 loads and stores them in one go).
  constexpr bool PF = sizeof(T) == 4 && RP == 2 && TXC > 0;
  constexpr bool PG = RP == 2 && TXC > 0;
  T ra[RP][6], rg[RP];
  auto fetch_vel = [&](int kk) {
    const int kc = min(max(kk, 0), nz - 1);
    const bool wz = kk < 0 || kk >= nz - 1;
    const size_t o = kc * layer;
    const T *ua = in.un + o, *ub = in.unm1 + o, *va = in.vn + o, *vb = in.vnm1 + o;
    const T *wa = in.wn + o, *wb = in.wnm1 + o;
    H.each_q([&](int q, int, unsigned off) {
      ra[q][0] = ld_at(ua, off);
      ra[q][2] = ld_at(va, off);
      ra[q][4] = wz ? (T)0 : ld_at(wa, off);
      ra[q][1] = f ? (T)0 : ld_at(ub, off);
      ra[q][3] = f ? (T)0 : ld_at(vb, off);
      ra[q][5] = (f || wz) ? (T)0 : ld_at(wb, off);
    });
  };
  // extrapolated velocities on layer kk from the fetched values: no-slip ghosts (twice the
  // wall velocity minus the adjacent layer) for u, v beyond the walls; w is zero on and beyond
  // the walls. The thread's own point (the tile's first) also leaves its level n-1 values in
  // prev_next, for the hat of that layer.
  auto put_vel = [&](int kk) {
    const int sl = (kk - K0 + 1) % 3;
    const T sg = (kk < 0 || kk >= nz) ? (T)-1 : (T)1;
    const T bu = kk < 0 ? (T)(2.0 * c.uwb[0]) : kk >= nz ? (T)(2.0 * c.uwt[0]) : (T)0;
    const T bv = kk < 0 ? (T)(2.0 * c.uwb[1]) : kk >= nz ? (T)(2.0 * c.uwt[1]) : (T)0;
    const bool wz = kk < 0 || kk >= nz - 1;
    H.each_q([&](int q, int e, unsigned) {
      // each value read once: u* = 2 u^n - u^{n-1} (u^n on the first step)
      const T un = ra[q][0], um = ra[q][1], vn = ra[q][2], vm = ra[q][3], wn = ra[q][4], wm = ra[q][5];
      sU[sl * HP + e] = bu + sg * (f ? un : (T)2 * un - um);
      sV[sl * HP + e] = bv + sg * (f ? vn : (T)2 * vn - vm);
      sW[sl * HP + e] = wz ? (T)0 : (f ? wn : (T)2 * wn - wm);
      if (q == 0) {
        prev_next[0] = um;
        prev_next[1] = vm;
        prev_next[2] = wm;
      }
    });
  };
  // without the prefetch each value is combined as it arrives (fewer live registers)
  auto load_vel = [&](int kk) {
    if constexpr (PF) {
      fetch_vel(kk);
      put_vel(kk);
    } else {
      const int sl = (kk - K0 + 1) % 3;
      const int kc = min(max(kk, 0), nz - 1);
      const T sg = (kk < 0 || kk >= nz) ? (T)-1 : (T)1;
      const T bu = kk < 0 ? (T)(2.0 * c.uwb[0]) : kk >= nz ? (T)(2.0 * c.uwt[0]) : (T)0;
      const T bv = kk < 0 ? (T)(2.0 * c.uwb[1]) : kk >= nz ? (T)(2.0 * c.uwt[1]) : (T)0;
      const bool wz = kk < 0 || kk >= nz - 1;
      const size_t o = kc * layer;
      const T *ua = in.un + o, *ub = in.unm1 + o, *va = in.vn + o, *vb = in.vnm1 + o;
      const T *wa = in.wn + o, *wb = in.wnm1 + o;
      H.each_q([&](int q, int e, unsigned off) {
        const T un = ld_at(ua, off), vn = ld_at(va, off), wn = wz ? (T)0 : ld_at(wa, off);
        const T um = f ? (T)0 : ld_at(ub, off), vm = f ? (T)0 : ld_at(vb, off);
        const T wm = (f || wz) ? (T)0 : ld_at(wb, off);
        sU[sl * HP + e] = bu + sg * (f ? un : (T)2 * un - um);
        sV[sl * HP + e] = bv + sg * (f ? vn : (T)2 * vn - vm);
        sW[sl * HP + e] = wz ? (T)0 : (f ? wn : (T)2 * wn - wm);
        if (q == 0) {
          prev_next[0] = um;
          prev_next[1] = vm;
          prev_next[2] = wm;
        }
      });
    }
  };
  auto fetch_g = [&](int kk) {
    const T* g = R.G_c + min(max(kk, 0), nz - 1) * layer;
    H.each_q([&](int q, int, unsigned off) { rg[q] = ld_at(g, off); });
  };
  auto put_g = [&](int kk) {
    const int sl = (kk - K0 + 1) & 3;
    H.each_q([&](int q, int e, unsigned) { sG[sl * HP + e] = rg[q]; });
  };
  auto load_g = [&](int kk) {
    if constexpr (PG) {
      fetch_g(kk);
      put_g(kk);
    } else {
      const int sl = (kk - K0 + 1) & 3;
      const T* g = R.G_c + min(max(kk, 0), nz - 1) * layer;
      H.each([&](int e, unsigned off) { sG[sl * HP + e] = ld_at(g, off); });
    }
  };
  load_vel(K0 - 1);
  load_vel(K0);
  T prev[3] = {prev_next[0], prev_next[1], prev_next[2]};  // own level n-1 u, v, w on layer k
  load_g(K0 - 1);
  load_g(K0);
  load_g(K0 + 1);
  if constexpr (PF) fetch_vel(K0 + 1);
  if constexpr (PG) fetch_g(K0 + 2);
  const int K1 = min(K0 + KB, nz);  // the last block of a column may march fewer layers
  // the own column's pressure, phi_c, mu_c and z-edge viscosities on layers k and k + 1 stay
  // in registers: each is read from memory once per layer
  const Field<T> Pg{in.pn, in.pnm1, nx, ny, nz, f};
  const Coarse<T> Phg{R.phi_c, nx, ny, nz}, Mug{R.mu_c, nx, ny, nz};
  const ZEdge<T> Exg{R.mu_xz, nx, ny}, Eyg{R.mu_yz, nx, ny};
  T ps0 = Pg.s(K0, j, i), pn0 = Pg.n(K0, j, i), ph0 = Phg.at(K0, j, i), mu0 = Mug.at(K0, j, i);
  T ex0 = Exg.at(K0, j, i), ey0 = Eyg.at(K0, j, i);
  for (int k = K0; k < K1; ++k) {
    if constexpr (PF)
      put_vel(k + 1);
    else
      load_vel(k + 1);
    if constexpr (PG)
      put_g(k + 2);
    else
      load_g(k + 2);
    // layer k + 1 (clamped on the top layer, where no term reads it); the edges have nz + 1
    const int ku = min(k + 1, nz - 1);
    const T ps1 = Pg.s(ku, j, i), pn1 = Pg.n(ku, j, i), ph1 = Phg.at(ku, j, i), mu1 = Mug.at(ku, j, i);
    const T ex1 = Exg.at(k + 1, j, i), ey1 = Eyg.at(k + 1, j, i);
    __syncthreads();
    // the next iteration's layers, in flight while this layer is formed
    if (k + 2 <= K1) {
      if constexpr (PF) fetch_vel(k + 2);
      if constexpr (PG) fetch_g(k + 3);
    }
    const int v0 = (k - K0) % 3, v1 = (k - K0 + 1) % 3, v2 = (k - K0 + 2) % 3;
    const RingV<T> Ur{{sU + v0 * HP, sU + v1 * HP, sU + v2 * HP}, k, X0, Y0, ys};
    const RingV<T> Vr{{sV + v0 * HP, sV + v1 * HP, sV + v2 * HP}, k, X0, Y0, ys};
    const RingV<T> Wr{{sW + v0 * HP, sW + v1 * HP, sW + v2 * HP}, k, X0, Y0, ys};
    const RingG<T> Gr{{sG + ((k - K0) & 3) * HP, sG + ((k - K0 + 1) & 3) * HP, sG + ((k - K0 + 2) & 3) * HP,
                       sG + ((k - K0 + 3) & 3) * HP},
                      k, X0, Y0, ys};
    const PolPre<T> Pp{{in.pol[0], in.pol[1], in.pol[2]}};
    const PCol<T> Pc{Pg, k, j, i, ps0, ps1, pn0, pn1};
    MomCtxG<T, RingV<T>, RingG<T>, PolPre<T>, PCol<T>, ACol<T, Coarse<T>>, ACol<T, ZEdge<T>>, PrevOwn<T>> m{
        Ur, Vr, Wr,
        Pc,
        Pc,
        Gr,
        {Phg, k, j, i, ph0, ph1},
        {Mug, k, j, i, mu0, mu1},
        {R.mu_xy, nx, ny, nz},
        {Exg, k, j, i, ex0, ex1},
        {Eyg, k, j, i, ey0, ey1},
        Pp,
                                     R,
                                     in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1,
                                     nx, ny, nz, f, VE ? 1 : 0,
                                     ihx, ihy, ihz,
                                     (T)c.inv_dt, (T)c.inv_re, (T)c.inv_rho0, (T)c.nu_m, (T)c.k_sigma, (T)c.c_j,
                                     PrevOwn<T>{{prev[0], prev[1], prev[2]}}};
    auto rhs = [&](const MomTerms<T>& t, T a) -> T {
      return -t.hat * m.inv_dt + t.adv + t.ri * t.jg + t.gpn * m.ir0 + (t.ri - m.ir0) * t.gps + m.nu_m * t.lap -
             m.inv_re * t.ri * t.pol - m.inv_re * t.ri * t.vis - m.k_sigma * t.ri * t.cap - a;
    };
    const int id = (k * ny + j) * nx + i;
    st_nt(ru + id, rhs(mom_u(m, k, j, i, id), (T)c.ax));
    st_nt(rv + id, rhs(mom_v(m, k, j, i, id), (T)c.ay));
    st_nt(rw + id, k == nz - 1 ? (T)0 : rhs(mom_w(m, k, j, i, id), (T)c.az));
    for (int a = 0; a < 3; ++a) prev[a] = prev_next[a];
    ps0 = ps1;
    pn0 = pn1;
    ph0 = ph1;
    mu0 = mu1;
    ex0 = ex1;
    ey0 = ey1;
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
                    T ihy, T ihz, T dt, T inv_wi, T one_m_beta, T gk, T c0, T c1, Walls<T> wl) {
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
  velocity_gradient(U, V, Wf, k, j, i, nz, ihx, ihy, ihz, L, wl);
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

// LDS view of coarse layers in a three-slot ring (slot (k - K0 + 3) mod 3) over a block's box
// (its tile with two cells of halo in x and y): at(k, j, i) for unwrapped global j, i inside
// the box.
template <typename T>
struct BoxRing {
  const T* base;
  int plane, K0, X0, Y0, BX;
  __device__ __forceinline__ T at(int k, int j, int i) const {
    return base[((k - K0 + 3) % 3) * plane + (j - Y0 + 2) * BX + (i - X0 + 2)];
  }
};

// Right-hand side RH of the stress equation (eqs. NS40-NS41 in stress form) at one cell, for
// all six components: t0 the cell's stress, S the LDS planes (component c at S + c * plane)
// holding the stress of the cell's layer at box index e (x neighbours e -+ 1, y neighbours e -+ BX),
// zm / zp the stress of the cells below and above (used only where lo / hi: no flux through
// a wall), L the velocity gradient and u-, u+, v-, v+, w-, w+ the face velocities.
template <typename T>
__device__ __forceinline__ void stress_rhs(const T t0[6], const T* S, int plane, int e, int BX,
                                           const T zm[6], const T zp[6], bool lo, bool hi,
                                           const T L[3][3], const T f[6], T ihx, T ihy, T ihz,
                                           T inv_wi, T omb, T gk, T rh[6]) {
  const T h = (T)0.5;
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int a = pairs[m][0], b = pairs[m][1];
    const T* q = S + m * plane;
    const T c = t0[m];
    const T fxp = f[1] * h * (c + q[e + 1]);
    const T fxm = f[0] * h * (q[e - 1] + c);
    const T fyp = f[3] * h * (c + q[e + BX]);
    const T fym = f[2] * h * (q[e - BX] + c);
    const T fzp = hi ? f[5] * h * (c + zp[m]) : (T)0;
    const T fzm = lo ? f[4] * h * (zm[m] + c) : (T)0;
    T r = -((fxp - fxm) * ihx + (fyp - fym) * ihy + (fzp - fzm) * ihz);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) r += L[cc][a] * t0[tidx(cc, b)] + t0[tidx(a, cc)] * L[cc][b];
    r += (omb * (L[a][b] + L[b][a]) - c) * inv_wi;
    if (gk != (T)0) {
      T tt = 0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) tt += t0[tidx(a, cc)] * t0[tidx(cc, b)];
      r -= gk * tt;
    }
    rh[m] = r;
  }
}

// Both stages of the RK2-TVD polymer update (eqs. NS42, NS44) with u^{n+1} fixed, in one
// z-marching pass over 3D grids, central advection: a block owns TX x TY columns and KB layers.
// Stage 1 gives tau^(1) on the tile and on the ring of cells around it whose tau^(1) the
// stage-2 advection of the tile reads (2 (TX + TY) cells per layer, recomputed by the
// neighbouring block too); tau^(1) stays in LDS (the layer being finished) and in registers
// (the cell's own column), and never goes to memory. LDS per block: tau^n of the stage-1 layer
// and tau^(1) of the stage-2 layer over the box (tile plus two cells of halo), and three-layer
// rings of u, v, w over the box, from which the velocity gradient of eq. NS41 is formed (the
// tile cell keeps its own for stage 2). Each thread loads at
// most RP box points.
template <typename T, int RP, int WPE, bool PF, int TXC = 0, int NT = kBlock>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
    k_polymer_rk2_zm(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
                     TauSet<T> tn, TauOut<T> tout, int nx, int ny, int nz, int KB, T ihx, T ihy,
                     T ihz, T dt, T inv_wi, T omb, T gk, Walls<T> wl) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TX = TXC > 0 ? TXC : (int)blockDim.x, TY = TXC > 0 ? NT / TXC : (int)blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int X0 = bx * TX, Y0 = by * TY, K0 = bz * KB;
  const int K1 = min(K0 + KB, nz);
  const int BX = TX + 4, BOX = BX * (TY + 4);
  const int tid = threadIdx.y * TX + threadIdx.x, nth = TX * TY;
  T* sTn = reinterpret_cast<T*>(smem);  // 6 planes: tau^n of the stage-1 layer
  T* sT1 = sTn + 6 * BOX;               // 6 planes: tau^(1) of the stage-2 layer
  T* sU = sT1 + 6 * BOX;                // 3-slot rings of u, v, w
  T* sV = sU + 3 * BOX;
  T* sW = sV + 3 * BOX;
  const BoxRing<T> Ur{sU, BOX, K0, X0, Y0, BX}, Vr{sV, BOX, K0, X0, Y0, BX}, Wr{sW, BOX, K0, X0, Y0, BX};
  const size_t layer = (size_t)nx * ny;
  // this thread's box points (own_first_point: point 0 is the thread's own column) and their
  // in-layer byte offsets
  int bpos[RP];
  unsigned off[RP];
#pragma unroll
  for (int q = 0; q < RP; ++q) {
    int hy = 0, hx = 0;
    const bool in = own_first_point<2, 2>(TX, TY, tid, q, hy, hx);
    bpos[q] = in ? hy * BX + hx : -1;
    off[q] = in ? (unsigned)(wrap(Y0 - 2 + hy, ny) * nx + wrap(X0 - 2 + hx, nx)) * (unsigned)sizeof(T) : 0u;
  }
  // own tile cell and, for the first 2 (TX + TY) threads, one ring cell
  const int i = X0 + threadIdx.x, j = Y0 + threadIdx.y;
  const int eo = (threadIdx.y + 2) * BX + threadIdx.x + 2;
  const unsigned oo = (unsigned)(j * nx + i) * (unsigned)sizeof(T);
  const bool has_h = tid < 2 * (TX + TY);
  int hi_ = X0, hj = Y0;
  if (tid < TX) {
    hi_ = X0 + tid;
    hj = Y0 - 1;
  } else if (tid < 2 * TX) {
    hi_ = X0 + tid - TX;
    hj = Y0 + TY;
  } else if (tid < 2 * TX + TY) {
    hi_ = X0 - 1;
    hj = Y0 + tid - 2 * TX;
  } else {
    hi_ = X0 + TX;
    hj = Y0 + tid - 2 * TX - TY;
  }
  const int eh = (hj - Y0 + 2) * BX + (hi_ - X0 + 2);
  const unsigned oh = (unsigned)(wrap(hj, ny) * nx + wrap(hi_, nx)) * (unsigned)sizeof(T);

  // Every access is the array's base plus a 32-bit byte offset (layer offset + in-layer
  // offset; the launcher keeps arrays below 4 GB), so that no 64-bit per-lane address is
  // formed or kept. With PF the box loads of the next layer are issued one layer ahead into
  // registers (FP32, which has the registers for it); otherwise they go straight to LDS.
  const unsigned lbytes = (unsigned)(layer * sizeof(T));
  T rt[PF ? RP : 1][6], rv[PF ? RP : 1][3];
  auto fetch_tau = [&](int m) {
    const unsigned o = (unsigned)m * lbytes;
#pragma unroll
    for (int q = 0; q < RP; ++q)
#pragma unroll
      for (int c = 0; c < 6; ++c) rt[PF ? q : 0][c] = bpos[q] >= 0 ? ld_at(tn.p[c], o + off[q]) : (T)0;
  };
  auto put_tau = [&]() {
#pragma unroll
    for (int q = 0; q < RP; ++q)
      if (bpos[q] >= 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) sTn[c * BOX + bpos[q]] = rt[q][c];
  };
  auto fetch_vel = [&](int l) {
    const unsigned o = (unsigned)l * lbytes;
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      rv[PF ? q : 0][0] = bpos[q] >= 0 ? ld_at(u, o + off[q]) : (T)0;
      rv[PF ? q : 0][1] = bpos[q] >= 0 ? ld_at(v, o + off[q]) : (T)0;
      rv[PF ? q : 0][2] = bpos[q] >= 0 ? ld_at(w, o + off[q]) : (T)0;
    }
  };
  auto put_vel = [&](int l) {
    const int sl = ((l - K0 + 3) % 3) * BOX;
#pragma unroll
    for (int q = 0; q < RP; ++q)
      if (bpos[q] >= 0) {
        sU[sl + bpos[q]] = rv[q][0];
        sV[sl + bpos[q]] = rv[q][1];
        sW[sl + bpos[q]] = rv[q][2];
      }
  };
  auto box_tau = [&](int m) {
    const unsigned o = (unsigned)m * lbytes;
#pragma unroll
    for (int q = 0; q < RP; ++q)
      if (bpos[q] >= 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) sTn[c * BOX + bpos[q]] = ld_at(tn.p[c], o + off[q]);
  };
  auto box_vel = [&](int l) {
    const unsigned o = (unsigned)l * lbytes;
    const int sl = ((l - K0 + 3) % 3) * BOX;
#pragma unroll
    for (int q = 0; q < RP; ++q)
      if (bpos[q] >= 0) {
        sU[sl + bpos[q]] = ld_at(u, o + off[q]);
        sV[sl + bpos[q]] = ld_at(v, o + off[q]);
        sW[sl + bpos[q]] = ld_at(w, o + off[q]);
      }
  };
  auto load_col = [&](int m, unsigned oc, T (&t)[6]) {
    const unsigned o = (unsigned)m * lbytes + oc;
#pragma unroll
    for (int c = 0; c < 6; ++c) t[c] = ld_at(tn.p[c], o);
  };
  // velocity gradient and face velocities (u-, u+, v-, v+, w-, w+) of a cell from the rings
  auto kinematics = [&](int m, int jj, int ii, T (&L)[3][3], T (&f)[6]) {
    velocity_gradient(Ur, Vr, Wr, m, jj, ii, nz, ihx, ihy, ihz, L, wl);
    f[0] = Ur.at(m, jj, ii - 1);
    f[1] = Ur.at(m, jj, ii);
    f[2] = Vr.at(m, jj - 1, ii);
    f[3] = Vr.at(m, jj, ii);
    f[4] = m > 0 ? Wr.at(m - 1, jj, ii) : (T)0;
    f[5] = m < nz - 1 ? Wr.at(m, jj, ii) : (T)0;
  };

  const int mlo = K0 > 0 ? K0 - 1 : 0;
  if (mlo > 0) box_vel(mlo - 1);
  box_vel(mlo);
  if constexpr (PF) {
    fetch_tau(mlo);
    if (mlo + 1 < nz) fetch_vel(mlo + 1);
  }
  // own column, carried up the march: tau^n of layer m - 1 (tA), tau^(1) of layers k - 1 and k
  // (t1p, t1c) and the kinematics of layer k (Lk, fk) for stage 2 at k = m - 1
  T tA[6], t1p[6], t1c[6], Lk[3][3], fk[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) tA[c] = t1p[c] = t1c[c] = fk[c] = (T)0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Lk[a][b] = (T)0;
  if (mlo > 0) load_col(mlo - 1, oo, tA);
  for (int m = mlo; m <= K1; ++m) {
    // tau^n of layer m and the velocities of layer m + 1 into LDS; the own column above
    T tB[6], tC[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) tC[c] = (T)0;
    if constexpr (PF) {
      // the own column's tau^n of layer m + 1 is the first point of that layer's box fetch
      if (m < nz) put_tau();
      if (m + 1 < nz) put_vel(m + 1);
      __syncthreads();
      if (m + 1 < nz) {
        fetch_tau(m + 1);
#pragma unroll
        for (int c = 0; c < 6; ++c) tC[c] = rt[0][c];
      }
      if (m + 2 < nz) fetch_vel(m + 2);
    } else {
      if (m < nz) box_tau(m);
      if (m + 1 < nz) box_vel(m + 1);
      if (m + 1 < nz) load_col(m + 1, oo, tC);
      __syncthreads();
    }
    // ---- stage 1 at layer m, own cell: tau^(1) = tau^n + dt RH(tau^n)
    T t1o[6], Lm[3][3], fm[6], rh[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) t1o[c] = tB[c] = (T)0;
    if (m < nz) {
#pragma unroll
      for (int c = 0; c < 6; ++c) tB[c] = sTn[c * BOX + eo];
      kinematics(m, j, i, Lm, fm);
      stress_rhs<T>(tB, sTn, BOX, eo, BX, tA, tC, m > 0, m < nz - 1, Lm, fm, ihx, ihy, ihz, inv_wi, omb, gk, rh);
#pragma unroll
      for (int c = 0; c < 6; ++c) t1o[c] = tB[c] + dt * rh[c];
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- stage 2 at layer k = m - 1: tau^{n+1} = tau^n / 2 + (tau^(1) + dt RH(tau^(1))) / 2
    const int k = m - 1;
    if (k >= K0) {
      stress_rhs<T>(t1c, sT1, BOX, eo, BX, t1p, t1o, k > 0, k < nz - 1, Lk, fk, ihx, ihy, ihz, inv_wi, omb, gk, rh);
      const unsigned o = (unsigned)k * lbytes + oo;
#pragma unroll
      for (int c = 0; c < 6; ++c) st_nt_at(tout.p[c], o, (T)0.5 * tA[c] + (T)0.5 * (t1c[c] + dt * rh[c]));
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- stage 1 at layer m, ring cell (needed only for stage 2 of this block's layers); its
    // column's tau^n above and below straight from memory
    T t1h[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) t1h[c] = (T)0;
    const bool ring = has_h && m >= K0 && m < K1;
    if (ring) {
      T hm[6], h0[6], hp[6], Lh[3][3], fh[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        hm[c] = hp[c] = (T)0;
        h0[c] = sTn[c * BOX + eh];
      }
      if (m > 0) load_col(m - 1, oh, hm);
      if (m < nz - 1) load_col(m + 1, oh, hp);
      kinematics(m, hj, hi_, Lh, fh);
      stress_rhs<T>(h0, sTn, BOX, eh, BX, hm, hp, m > 0, m < nz - 1, Lh, fh, ihx, ihy, ihz, inv_wi, omb, gk, rh);
#pragma unroll
      for (int c = 0; c < 6; ++c) t1h[c] = h0[c] + dt * rh[c];
    }
    __syncthreads();
    // tau^(1) of layer m becomes the stage-2 layer of the next step
    if (m < nz) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sT1[c * BOX + eo] = t1o[c];
      if (ring)
#pragma unroll
        for (int c = 0; c < 6; ++c) sT1[c * BOX + eh] = t1h[c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      t1p[c] = t1c[c];
      t1c[c] = t1o[c];
      fk[c] = fm[c];
      tA[c] = tB[c];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) Lk[a][b] = Lm[a][b];
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
  // FP32: 64 x 8 columns (512 threads, two blocks per CU) where the grid allows: the halo tile
  // rows span four full cache lines plus two halo sectors instead of one plus two (at 256 x 256
  // x 128: momentum with its polymer divergence 434 -> 397 us). FP64 keeps 32 x 8: at three
  // waves per SIMD a CU holds one 512-thread block, against three of 256.
  const bool wide = sizeof(T) == 4 && c.nx >= 64 && c.ny >= 8;
  const int TX = wide ? 64 : (c.nx < 32 ? c.nx : 32);
  const int TY = wide ? 8 : (c.ny < kBlock / TX ? c.ny : kBlock / TX);
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
    // the face divergences of the weighted polymer stress first (15 LDS tile slots)
    const size_t shp = (size_t)15 * HP * sizeof(T);
    if (need <= 2)
      if (wide)
        go(k_polymer_div_zm<T, 2, 64, 512>, shp, in, (const T*)r.phi_c, k.first, c.nx, c.ny, c.nz);
      else if (TX == 32 && TY == 8)
        go(k_polymer_div_zm<T, 2, 32>, shp, in, (const T*)r.phi_c, k.first, c.nx, c.ny, c.nz);
      else
        go(k_polymer_div_zm<T, 2>, shp, in, (const T*)r.phi_c, k.first, c.nx, c.ny, c.nz);
    else
      go(k_polymer_div_zm<T, 4>, shp, in, (const T*)r.phi_c, k.first, c.nx, c.ny, c.nz);
  }
  const size_t shm = (size_t)13 * HP * sizeof(T);
#define DRPF_MOM(VE, RP, TXC, NT) go(k_momentum_rhs_zm<T, VE, RP, TXC, NT>, shm, in, r, ru, rv, rw, k, c.nx, c.ny, c.nz)
  // the 32 x 8 tile with its shape at compile time
  const bool t32 = TX == 32 && TY == 8;
  if (in.viscoelastic) {
    if (wide) DRPF_MOM(true, 2, 64, 512); else if (t32) DRPF_MOM(true, 2, 32, kBlock);
    else if (need <= 2) DRPF_MOM(true, 2, 0, kBlock); else DRPF_MOM(true, 4, 0, kBlock);
  } else {
    if (wide) DRPF_MOM(false, 2, 64, 512); else if (t32) DRPF_MOM(false, 2, 32, kBlock);
    else if (need <= 2) DRPF_MOM(false, 2, 0, kBlock); else DRPF_MOM(false, 4, 0, kBlock);
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
  const Walls<T> wl = walls_of<T>(k);
  if (k.advection == 1)
    hipLaunchKernelGGL((k_polymer_stage<T, true>), L.grid, L.block, 0, st, u, v, w, tn, ti, to, c.nx, c.ny,
                       c.nz, (T)c.ihx, (T)c.ihy, (T)c.ihz, (T)k.dt, (T)k.inv_wi, (T)(1.0 - k.beta), gk, (T)c0,
                       (T)c1, wl);
  else
    hipLaunchKernelGGL((k_polymer_stage<T, false>), L.grid, L.block, 0, st, u, v, w, tn, ti, to, c.nx, c.ny,
                       c.nz, (T)c.ihx, (T)c.ihy, (T)c.ihz, (T)k.dt, (T)k.inv_wi, (T)(1.0 - k.beta), gk, (T)c0,
                       (T)c1, wl);
  return hipGetLastError();
}

template <typename T>
bool polymer_rk2_fused(const Dims& c, const StepConsts& k) {
  // 3D, central advection, and arrays addressed by 32-bit byte offsets
  return c.ny > 1 && k.advection == 0 && c.cells() * sizeof(T) < ((size_t)1 << 32);
}

template <typename T>
hipError_t launch_polymer_rk2(const Dims& c, const StepConsts& k, const T* u, const T* v, const T* w,
                              const T* const tau_n[6], T* const tau_out[6], hipStream_t st) {
  if (!polymer_rk2_fused<T>(c, k)) return hipErrorInvalidValue;
  TauSet<T> tn;
  TauOut<T> to;
  for (int m = 0; m < 6; ++m) {
    tn.p[m] = tau_n[m];
    to.p[m] = tau_out[m];
  }
  // 64 x 8 columns (512 threads, two blocks per CU) where the grid allows: the two-cell halo box
  // is 1.59x the tile instead of 1.69x and a box row is four cache lines plus two halo sectors
  // instead of one plus two, so fewer halo bytes are fetched per cell (at 256 x 256 x 128: RK2
  // march 223 -> 206 us FP32, 471 -> 415 us FP64)
  const bool wide = c.nx >= 64 && c.ny >= 8;
  const int TX = wide ? 64 : (c.nx < 32 ? c.nx : 32);
  const int TY = wide ? 8 : (c.ny < kBlock / TX ? c.ny : kBlock / TX);
  const int cols = (c.nx / TX) * (c.ny / TY);
  const int BOX = (TX + 4) * (TY + 4);
  const int need = (BOX + TX * TY - 1) / (TX * TY);
  if (need > 4 || 2 * (TX + TY) > TX * TY) return hipErrorInvalidConfiguration;
  const size_t shm = (size_t)21 * BOX * sizeof(T);
  const T gk = (T)(k.giesekus == 0.0 ? 0.0 : k.giesekus / (1.0 - k.beta));
  const Walls<T> wl = walls_of<T>(k);
  auto go = [&](auto kernel) {
    const int KB = march_layers(kernel, TX * TY, shm, cols, c.nz);
    const dim3 grid(c.nx / TX, c.ny / TY, (c.nz + KB - 1) / KB);
    hipLaunchKernelGGL(kernel, grid, dim3(TX, TY), shm, st, u, v, w, tn, to, c.nx, c.ny, c.nz, KB, (T)c.ihx,
                       (T)c.ihy, (T)c.ihz, (T)k.dt, (T)k.inv_wi, (T)(1.0 - k.beta), gk, wl);
  };
  // registers: with the 32 x 8 or 64 x 8 shape at compile time FP32 fits four waves per SIMD
  // (128 VGPRs) and FP64 two (202 / 240), without spills; with the shape at run time FP32 takes 2 waves per SIMD
  // (226 VGPRs) and FP64 1 (at 2 waves it spills to scratch: 2.5x the algorithmic bytes on the
  // C5 grid and slower, 864 against 731 us)
  constexpr int WPE = sizeof(T) == 4 ? 2 : 1;
  constexpr int WPE32 = sizeof(T) == 4 ? 4 : 2;
  constexpr bool PF = sizeof(T) == 4;
  if (wide)
    go(k_polymer_rk2_zm<T, 2, WPE32, PF, 64, 512>);
  else if (TX == 32 && TY == 8)
    go(k_polymer_rk2_zm<T, 2, WPE32, PF, 32>);
  else if (need <= 2)
    go(k_polymer_rk2_zm<T, 2, WPE, PF>);
  else
    go(k_polymer_rk2_zm<T, 4, WPE, PF>);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template bool polymer_rk2_fused<T>(const Dims&, const StepConsts&);                            \
  template hipError_t launch_polymer_rk2<T>(const Dims&, const StepConsts&, const T*, const T*,   \
                                            const T*, const T* const[6], T* const[6], hipStream_t); \
  template hipError_t launch_momentum_rhs<T>(const Dims&, const StepConsts&, NsIn<T>,             \
                                             Restricted<T>, T*, T*, T*, hipStream_t);             \
  template hipError_t launch_polymer_stage<T>(const Dims&, const StepConsts&, const T*, const T*, \
                                              const T*, const T* const[6], const T* const[6],     \
                                              T* const[6], double, double, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
