// Fine-grid (phase-field) stencils and the dual-grid transfers.
//
//   ch_rhs      -- right-hand side of the fused Cahn-Hilliard solve. With L_N the
//                  Laplacian with zero-flux ghosts and b the wetting data (the static-angle
//                  condition of eqs. NS15-NS16 with D_w = 0, evaluated at phi*, eq. NS34),
//                  eq. NS25 reads (L_N - c_psi)(L_N + alpha) phi^{n+1} = Q - L_N b with Q of
//                  eq. NS28. This kernel writes Q - L_N b; the spectral pass then applies
//                  the two Helmholtz inverses back to back (eqs. NS26-NS27). The fine face
//                  velocities come from the coarse ones by eq. dual1 on the fly.
//   restrict_g  -- chemical potential G^{n+1} = Cn^2 [-L_w phi + (S/Cn^2)(phi - phi*) +
//                  f(phi*)] (the bracket of eq. NS25 times the mixing energy), restriction of
//                  phi and G to coarse centres / faces / edges (eq. dual2) and the mixture
//                  properties there (eq. dual3): 1/rho at faces, solvent viscosity at centres
//                  and edges. A block marches up a column of coarse cells with rings of
//                  fine phi^{n+1} and G layers in LDS; G is evaluated once per fine cell and
//                  every thread sums its coarse cell's 2x2x2 groups from LDS.
//   prolong, restrict -- the standalone transfer operators (eqs. dual1, dual2).
#include "fine.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;

// Right-hand side of the fused CH solve, z-marching: a block owns TX x TY fine columns and
// KB consecutive layers. Rings of three layers of phi* and w* (with a one-cell x/y halo) live
// in LDS; each thread walks up its column, so the x/y neighbours come from LDS, the z
// neighbours from the ring, and the coarse velocities of eq. dual1 are reloaded only when
// the column enters a new coarse layer.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_ch_rhs(const T* __restrict__ phin, const T* __restrict__ phinm1, Prolonged<T> pv,
             T* __restrict__ out, int nx, int ny, int nz, int KB, T ihx, T ihy, T ihz,
             StepConsts c) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TX = blockDim.x, TY = blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int X0 = bx * TX, Y0 = by * TY, K0 = bz * KB;
  const int HX = TX + 2, HY = TY + 2, HP = HX * HY;
  T* sP = reinterpret_cast<T*>(smem);  // 3 slots of phi*
  T* sW = sP + 3 * HP;                 // 3 slots of w* = f(phi*) - (S/Cn^2) phi*
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * TX + tx, nth = TX * TY;
  const int I = X0 + tx, J = Y0 + ty;
  const bool first = c.first != 0;
  const T icn2 = (T)c.inv_cn2, sc = (T)c.s_cn2;
  auto load_layer = [&](int Kl, int slot) {
    const int Kc = min(max(Kl, 0), nz - 1);  // beyond a wall: zero-flux ghost = adjacent layer
    for (int e = tid; e < HP; e += nth) {
      const int hy = e / HX, hx = e - hy * HX;
      const int id = (Kc * ny + wrap(Y0 - 1 + hy, ny)) * nx + wrap(X0 - 1 + hx, nx);
      const T a = phin[id];
      const T p = first ? a : (T)2 * a - phinm1[id];
      sP[slot * HP + e] = p;
      sW[slot * HP + e] = (p * p * p - p) * icn2 - sc * p;
    }
  };
  int sm = 0, s0 = 1, sp = 2;
  load_layer(K0 - 1, sm);
  load_layer(K0, s0);
  // coarse column of this fine column (eq. dual1)
  const int ry = pv.ry;
  const int ic = I >> 1, icw = wrap(ic - 1, pv.cnx);
  const int jc = ry == 2 ? (J >> 1) : 0, jcw = ry == 2 ? wrap(jc - 1, pv.cny) : 0;
  const int cplane = pv.cnx * pv.cny;
  const int cu0 = jc * pv.cnx + ic, cu1 = jc * pv.cnx + icw;
  const int cv1 = jcw * pv.cnx + ic;
  const T ihx2 = ihx * ihx, ihy2 = ihy * ihy, ihz2 = ihz * ihz, h = (T)0.5;
  const T gb = (T)c.g_bot * ihz, gt = (T)c.g_top * ihz;
  T ufp = 0, ufm = 0, vfp = 0, vfm = 0, wk = 0, wkm = 0;
  int kcur = -1;
  for (int K = K0; K < K0 + KB; ++K) {
    load_layer(K + 1, sp);
    const int k = K >> 1;
    if (k != kcur) {
      kcur = k;
      const int o = k * cplane;
      const T ua = pv.star(pv.un, pv.unm1, o + cu0), ub = pv.star(pv.un, pv.unm1, o + cu1);
      const bool iodd = I & 1;
      ufp = iodd ? ua : h * (ub + ua);
      ufm = iodd ? h * (ub + ua) : ub;
      const T va = pv.star(pv.vn, pv.vnm1, o + cu0);
      if (ry == 2) {
        const T vb = pv.star(pv.vn, pv.vnm1, o + cv1);
        const bool jodd = J & 1;
        vfp = jodd ? va : h * (vb + va);
        vfm = jodd ? h * (vb + va) : vb;
      } else {
        vfp = vfm = va;
      }
      wk = k < pv.cnz - 1 ? pv.star(pv.wn, pv.wnm1, o + cu0) : (T)0;
      wkm = k > 0 ? pv.star(pv.wn, pv.wnm1, o - cplane + cu0) : (T)0;
    }
    // fine z faces K (above) and K-1 (below); the walls carry zero flux
    const T wfp = K == nz - 1 ? (T)0 : ((K & 1) ? wk : h * (wkm + wk));
    const T wfm = K == 0 ? (T)0 : ((K & 1) ? h * (wkm + wk) : wkm);
    __syncthreads();
    const int c0 = (ty + 1) * HX + (tx + 1);
    const T* P0 = sP + s0 * HP;
    const T* W0 = sW + s0 * HP;
    const T p0 = P0[c0], pxp = P0[c0 + 1], pxm = P0[c0 - 1], pyp = P0[c0 + HX], pym = P0[c0 - HX];
    const T pzp = sP[sp * HP + c0], pzm = sP[sm * HP + c0];
    const T w0 = W0[c0];
    const T lapw = (W0[c0 + 1] - 2 * w0 + W0[c0 - 1]) * ihx2 + (W0[c0 + HX] - 2 * w0 + W0[c0 - HX]) * ihy2 +
                   (sW[sp * HP + c0] - 2 * w0 + sW[sm * HP + c0]) * ihz2;
    const T adv = (ufp * h * (p0 + pxp) - ufm * h * (pxm + p0)) * ihx +
                  (vfp * h * (p0 + pyp) - vfm * h * (pym + p0)) * ihy +
                  (wfp * h * (p0 + pzp) - wfm * h * (pzm + p0)) * ihz;
    // wetting data b = g(phi*) / hz on the wall-adjacent layers, and L_N b
    auto bval = [&](int kk, T p) -> T {
      T b = 0;
      if (kk == 0) b += gb * ((T)1 - p * p);
      if (kk == nz - 1) b += gt * ((T)1 - p * p);
      return b;
    };
    T lapb = 0;
    if (K == 0 || K == nz - 1) {
      const T b0 = bval(K, p0);
      lapb = (bval(K, pxp) - 2 * b0 + bval(K, pxm)) * ihx2 + (bval(K, pyp) - 2 * b0 + bval(K, pym)) * ihy2;
      const T bup = K + 1 < nz ? bval(K + 1, pzp) : b0;
      const T bdn = K > 0 ? bval(K - 1, pzm) : b0;
      lapb += (bup - 2 * b0 + bdn) * ihz2;
    } else {
      if (K == 1) lapb += bval(0, pzm) * ihz2;
      if (K == nz - 2) lapb += bval(nz - 1, pzp) * ihz2;
    }
    const int id = (K * ny + J) * nx + I;
    const T phat = first ? phin[id] : (T)2 * phin[id] - (T)0.5 * phinm1[id];
    const T q = (T)c.pe_cn2 * (phat * (T)c.inv_dt - adv) + lapw;
    out[id] = q - lapb;
    __syncthreads();
    const int t = sm;
    sm = s0;
    s0 = sp;
    sp = t;
  }
}


// Chemical potential, restriction and properties, z-marching: a block owns CX x CY coarse
// columns and KB coarse layers. A ring of six fine layers of phi^{n+1} (one-cell halo) and a
// ring of four fine layers of G live in LDS, indexed by the clamped fine layer modulo the
// ring size; stepping one coarse layer up loads two new phi layers and evaluates G on two
// new layers (the shared face layer is kept). The block has 2 CY rows of threads: all of them
// load tiles and evaluate G; for the restricted sums the lower CY rows form the phi-derived
// outputs and the upper CY rows the G-derived ones of the same coarse cells. The global loads
// of the next layers are issued into registers before the sums and written to LDS after them,
// so that their latency overlaps the arithmetic.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_restrict_g(const T* __restrict__ phinew, const T* __restrict__ phin,
                 const T* __restrict__ phinm1, Restricted<T> r, int fnx, int fny, int fnz,
                 T fihx, T fihy, T fihz, int cnx, int cny, int cnz, int ry, int KB,
                 StepConsts c) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int RMAX = 6;  // per-thread share of a tile: PP, GP <= RMAX * threads (launcher)
  const int CX = blockDim.x, CY = blockDim.y / 2;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i0 = bx * CX, j0 = by * CY, k0 = bz * KB;
  const int GX = 2 * CX + 1, GY = ry * CY + 1, GP = GX * GY;
  const int PX = GX + 2, PY = GY + 2, PP = PX * PY;
  const int X0 = 2 * i0, Y0 = ry * j0;
  T* sP = reinterpret_cast<T*>(smem);  // 6 slots of phi^{n+1}
  T* sG = sP + 6 * PP;                 // 4 slots of G
  const int tid = threadIdx.y * CX + threadIdx.x;
  const int nth = CX * blockDim.y;
  const bool first = c.first != 0;
  const T ihx2 = fihx * fihx, ihy2 = fihy * fihy, ihz2 = fihz * fihz;
  const T cn2 = (T)c.cn2, S = (T)c.S;
  const T gb = (T)c.g_bot * fihz, gt = (T)c.g_top * fihz;
  auto kc = [&](int Kf) { return min(max(Kf, 0), fnz - 1); };
  auto pidx = [&](int K, int e) {
    const int py = e / PX, px = e - py * PX;
    return (K * fny + wrap(Y0 - 1 + py, fny)) * fnx + wrap(X0 - 1 + px, fnx);
  };
  auto gidx = [&](int K, int e) {
    const int gy = e / GX, gx = e - gy * GX;
    return (K * fny + wrap(Y0 + gy, fny)) * fnx + wrap(X0 + gx, fnx);
  };
  auto loadP = [&](int Kf) {
    const int K = kc(Kf);
    T* dst = sP + (K % 6) * PP;
    for (int e = tid; e < PP; e += nth) dst[e] = phinew[pidx(K, e)];
  };
  // G on fine layer Kf from the LDS ring of phi^{n+1}; phi* of the tile points given
  auto computeG_with = [&](int Kf, const T* psr) {
    const int K = kc(Kf);
    const T* Pm = sP + (kc(K - 1) % 6) * PP;
    const T* P0 = sP + (K % 6) * PP;
    const T* Pp = sP + (kc(K + 1) % 6) * PP;
    T* dst = sG + (K % 4) * GP;
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const int e = tid + q * nth;
      if (e < GP) {
        const int gy = e / GX, gx = e - gy * GX;
        const int m = (gy + 1) * PX + gx + 1;
        const T p = P0[m];
        const T lap = (P0[m + 1] - 2 * p + P0[m - 1]) * ihx2 + (P0[m + PX] - 2 * p + P0[m - PX]) * ihy2 +
                      (Pp[m] - 2 * p + Pm[m]) * ihz2;
        const T ps = psr[q];
        T b = 0;
        if (K == 0) b += gb * ((T)1 - ps * ps);
        if (K == fnz - 1) b += gt * ((T)1 - ps * ps);
        dst[e] = -cn2 * (lap + b) + S * (p - ps) + ps * ps * ps - ps;
      }
    }
  };
  auto load_ps = [&](int Kf, T* psr) {
    const int K = kc(Kf);
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const int e = tid + q * nth;
      if (e < GP) {
        const int id = gidx(K, e);
        const T an = phin[id];
        psr[q] = first ? an : (T)2 * an - phinm1[id];
      }
    }
  };
  {
    T ps0[RMAX], ps1[RMAX], ps2[RMAX];
    for (int Kf = 2 * k0 - 1; Kf <= 2 * k0 + 3; ++Kf) loadP(Kf);
    load_ps(2 * k0, ps0);
    load_ps(2 * k0 + 1, ps1);
    load_ps(2 * k0 + 2, ps2);
    __syncthreads();
    computeG_with(2 * k0, ps0);
    computeG_with(2 * k0 + 1, ps1);
    computeG_with(2 * k0 + 2, ps2);
    __syncthreads();
  }
  const int tx = threadIdx.x;
  const bool upper = threadIdx.y >= CY;
  const int ty = upper ? threadIdx.y - CY : threadIdx.y;
  const int i = i0 + tx, j = j0 + ty;
  const T r1 = (T)c.rho1, r2 = (T)c.rho2, m1 = (T)c.mu1, m2 = (T)c.mu2, hf = (T)0.5;
  auto rinv = [&](T ph) { return (T)1 / (hf * ((T)1 + ph) * r1 + hf * ((T)1 - ph) * r2); };
  auto mu = [&](T ph) { return hf * ((T)1 + ph) * m1 + hf * ((T)1 - ph) * m2; };
  const int plane = cnx * cny;
  const int ndy = ry + 1;
  for (int k = k0; k < k0 + KB; ++k) {
    const bool more = k + 1 < k0 + KB;
    // prefetch: phi^{n+1} on fine layers 2k+4, 2k+5 and phi* on 2k+3, 2k+4
    T pf4[RMAX], pf5[RMAX], ps3[RMAX], ps4[RMAX];
    if (more) {
      const int K4 = kc(2 * k + 4), K5 = kc(2 * k + 5);
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        const int e = tid + q * nth;
        if (e < PP) {
          pf4[q] = phinew[pidx(K4, e)];
          pf5[q] = phinew[pidx(K5, e)];
        }
      }
      load_ps(2 * k + 3, ps3);
      load_ps(2 * k + 4, ps4);
    }
    // Separable sums of the tensor-product rule: per z layer and y row, x sums over the
    // centre pair (dx 0,1) and the face pair (dx 1,2); then y pairs, then z pairs. The 1/8
    // weight is applied once at the end (a centre-located y axis without refinement counts
    // its single cell twice). Lower rows: phi (src sP, ring 6); upper rows: G (sG, ring 4).
    {
      T z_[3][4];  // per dz: [YcXc, YcXf, YfXc, YfXf]
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const int K = kc(2 * k + dz);
        T xc[3], xf[3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int gy = ry * ty + (dy < ndy ? dy : 0);
          const T* pr = upper ? sG + (K % 4) * GP + gy * GX + 2 * tx
                              : sP + (K % 6) * PP + (gy + 1) * PX + 2 * tx + 1;
          xc[dy] = pr[0] + pr[1];
          xf[dy] = pr[1] + pr[2];
        }
        if (ry == 2) {
          z_[dz][0] = xc[0] + xc[1];
          z_[dz][1] = xf[0] + xf[1];
          z_[dz][2] = xc[1] + xc[2];
          z_[dz][3] = xf[1] + xf[2];
        } else {
          z_[dz][0] = (T)2 * xc[0];
          z_[dz][1] = (T)2 * xf[0];
          z_[dz][2] = xc[0] + xc[1];
          z_[dz][3] = xf[0] + xf[1];
        }
      }
      const T e8 = (T)0.125;
      const int id = (k * cny + j) * cnx + i;
      if (upper) {
        r.G_c[id] = e8 * (z_[0][0] + z_[1][0]);
        r.G_x[id] = e8 * (z_[0][1] + z_[1][1]);
        r.G_y[id] = e8 * (z_[0][2] + z_[1][2]);
        r.G_z[id] = e8 * (z_[1][0] + z_[2][0]);
      } else {
        const T phic = e8 * (z_[0][0] + z_[1][0]);
        r.phi_c[id] = phic;
        r.ri_x[id] = rinv(e8 * (z_[0][1] + z_[1][1]));
        r.ri_y[id] = rinv(e8 * (z_[0][2] + z_[1][2]));
        r.ri_z[id] = rinv(e8 * (z_[1][0] + z_[2][0]));
        r.mu_c[id] = mu(phic);
        r.mu_xy[id] = mu(e8 * (z_[0][3] + z_[1][3]));
        // z-edge arrays carry nz + 1 layers: layer k + 1 is the edge at z = (k + 1) hz
        r.mu_xz[id + plane] = mu(e8 * (z_[1][1] + z_[2][1]));
        r.mu_yz[id + plane] = mu(e8 * (z_[1][2] + z_[2][2]));
        if (k == 0) {
          r.mu_xz[id] = mu((T)0.25 * z_[0][1]);
          r.mu_yz[id] = mu((T)0.25 * z_[0][2]);
        }
      }
    }
    if (more) {
      // fine phi layers 2k+4, 2k+5 replace 2k-2, 2k-1; G on 2k+3, 2k+4 replaces 2k-1, 2k
      const int K4 = kc(2 * k + 4), K5 = kc(2 * k + 5);
      T* d4 = sP + (K4 % 6) * PP;
      T* d5 = sP + (K5 % 6) * PP;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        const int e = tid + q * nth;
        if (e < PP) {
          d4[e] = pf4[q];
          d5[e] = pf5[q];
        }
      }
      __syncthreads();
      computeG_with(2 * k + 3, ps3);
      computeG_with(2 * k + 4, ps4);
      __syncthreads();
    }
  }
}
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_prolong(T* __restrict__ uf, T* __restrict__ vf, T* __restrict__ wf, int fnx, int fny,
              Prolonged<T> pv) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  const int K = blockIdx.z;
  const size_t id = ((size_t)K * fny + J) * fnx + I;
  uf[id] = pv.uf(K, J, I);
  vf[id] = pv.vf(K, J, I);
  wf[id] = pv.wf(K, J, I);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_restrict(const T* __restrict__ f, T* __restrict__ out, int fnx, int fny, int fnz, int cnx,
               int cny, int ry, int lx, int ly, int lz) {
  // lx/ly/lz: 0 centre-located, 1 face-located along that axis. A face-located z output has
  // cnz + 1 layers; layer m is the face at z = m hz (m = 0 the bottom wall).
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int m = blockIdx.z;
  const FineView<T> F{f, fnx, fny, fnz};
  int xs[2], ys[2], zs[2];
  double wy[2];
  if (lx) { xs[0] = 2 * i + 1; xs[1] = 2 * i + 2; } else { xs[0] = 2 * i; xs[1] = 2 * i + 1; }
  if (ry == 2) {
    if (ly) { ys[0] = 2 * j + 1; ys[1] = 2 * j + 2; } else { ys[0] = 2 * j; ys[1] = 2 * j + 1; }
    wy[0] = wy[1] = 0.5;
  } else {
    ys[0] = j;
    ys[1] = j + 1;
    wy[0] = ly ? 0.5 : 1.0;
    wy[1] = ly ? 0.5 : 0.0;
  }
  if (lz) {
    zs[0] = min(max(2 * m - 1, 0), fnz - 1);
    zs[1] = min(max(2 * m, 0), fnz - 1);
  } else {
    zs[0] = 2 * m;
    zs[1] = 2 * m + 1;
  }
  double s = 0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int d = 0; d < 2; ++d) s += 0.25 * wy[b] * (double)F.at(zs[a], ys[b], xs[d]);
  out[((size_t)m * cny + j) * cnx + i] = (T)s;
}

}  // namespace

template <typename T>
hipError_t launch_ch_rhs(const Dims& f, const Dims& c, const StepConsts& k, ChIn<T> in, T* rhs,
                         hipStream_t st) {
  Prolonged<T> pv{in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1, c.nx, c.ny, c.nz,
                  c.ny == 1 ? 1 : 2, k.first};
  int TX, TY;
  if (f.ny == 1) {
    TX = f.nx < 256 ? f.nx : 256;
    TY = 1;
  } else {
    TX = f.nx < 64 ? f.nx : 64;
    TY = f.ny < 4 ? f.ny : 4;
  }
  const int tiles = (f.nx / TX) * (f.ny / TY);
  int KB = 16;
  while (KB > 2 && (f.nz / KB) * tiles < 1024) KB >>= 1;
  if (KB > f.nz) KB = f.nz;
  const size_t shm = (size_t)6 * (TX + 2) * (TY + 2) * sizeof(T);
  hipLaunchKernelGGL(k_ch_rhs<T>, dim3(f.nx / TX, f.ny / TY, f.nz / KB), dim3(TX, TY, 1), shm, st,
                     in.phin, in.phinm1, pv, rhs, f.nx, f.ny, f.nz, KB, (T)f.ihx, (T)f.ihy, (T)f.ihz, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_g(const Dims& f, const Dims& c, const StepConsts& k, const T* phinew,
                             const T* phin, const T* phinm1, Restricted<T> r, hipStream_t st) {
  const int ry = c.ny == 1 ? 1 : 2;
  int CX, CY;
  if (ry == 2) {
    CX = c.nx < 32 ? c.nx : 32;
    CY = c.ny < 4 ? c.ny : 4;
  } else {
    CX = c.nx < 128 ? c.nx : 128;
    CY = 1;
  }
  // coarse layers per block: the z march amortises the fine z halo; keep >= ~1024 blocks
  const int tiles = (c.nx / CX) * (c.ny / CY);
  int KB = 8;
  while (KB > 1 && (c.nz / KB) * tiles < 1024) KB >>= 1;
  if (KB > c.nz) KB = c.nz;
  const int GX = 2 * CX + 1, GY = ry * CY + 1;
  // the kernel keeps at most 6 tile points per thread in registers
  if ((GX + 2) * (GY + 2) > 6 * 2 * CX * CY || GX * GY > 6 * 2 * CX * CY) return hipErrorInvalidConfiguration;
  const size_t shm = (size_t)(6 * (GX + 2) * (GY + 2) + 4 * GX * GY) * sizeof(T);
  hipLaunchKernelGGL(k_restrict_g<T>, dim3(c.nx / CX, c.ny / CY, c.nz / KB), dim3(CX, 2 * CY, 1), shm, st,
                     phinew, phin, phinm1, r, f.nx, f.ny, f.nz, (T)f.ihx, (T)f.ihy, (T)f.ihz, c.nx,
                     c.ny, c.nz, ry, KB, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Dims& f, const Dims& c, const T* u, const T* v, const T* w, T* uf,
                          T* vf, T* wf, hipStream_t st) {
  // first = 1: the star extrapolation reduces to the given level
  Prolonged<T> pv{u, u, v, v, w, w, c.nx, c.ny, c.nz, c.ny == 1 ? 1 : 2, 1};
  const Launch3 L = launch3(f.nx, f.ny, f.nz);
  hipLaunchKernelGGL(k_prolong<T>, L.grid, L.block, 0, st, uf, vf, wf, f.nx, f.ny, pv);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const Dims& f, const Dims& c, const T* fine, T* coarse, int location,
                           hipStream_t st) {
  int lx = 0, ly = 0, lz = 0;
  switch (location) {
    case 0: break;
    case 1: lx = 1; break;
    case 2: ly = 1; break;
    case 3: lz = 1; break;
    case 4: lx = ly = 1; break;
    case 5: lx = lz = 1; break;
    case 6: ly = lz = 1; break;
    default: return hipErrorInvalidValue;
  }
  const int nzo = lz ? c.nz + 1 : c.nz;
  const Launch3 L = launch3(c.nx, c.ny, nzo);
  hipLaunchKernelGGL(k_restrict<T>, L.grid, L.block, 0, st, fine, coarse, f.nx, f.ny, f.nz, c.nx,
                     c.ny, c.ny == 1 ? 1 : 2, lx, ly, lz);
  return hipGetLastError();
}

#define INST(T)                                                                                   \
  template hipError_t launch_ch_rhs<T>(const Dims&, const Dims&, const StepConsts&, ChIn<T>, T*, \
                                       hipStream_t);                                              \
  template hipError_t launch_restrict_g<T>(const Dims&, const Dims&, const StepConsts&, const T*, \
                                           const T*, const T*, Restricted<T>, hipStream_t);       \
  template hipError_t launch_prolong<T>(const Dims&, const Dims&, const T*, const T*, const T*,   \
                                        T*, T*, T*, hipStream_t);                                 \
  template hipError_t launch_restrict<T>(const Dims&, const Dims&, const T*, T*, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
