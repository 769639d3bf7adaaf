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
//   g_single, props_single -- the same set when the phase field lives on the flow grid
//                  (single resolution): G and phi at the cells, then face and edge means.
//   prolong, restrict -- the standalone transfer operators (eqs. dual1, dual2).
#include "fine.hpp"
#include "weno.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;

// Right-hand side of the fused CH solve, z-marching: a block owns TX x TY fine columns and
// KB consecutive layers. Rings of three layers of phi* and w* (with a one-cell x/y halo) live
// in LDS; each thread walks up its column, so the x/y neighbours come from LDS and the z
// neighbours from the ring. Each thread owns at most R points of the halo tile (in-layer
// offsets computed once); the tile of the layer after next and the centre values of the next
// layer are loaded one step ahead into registers, so that their latency overlaps the
// arithmetic of the current layer. The coarse velocities of eq. dual1 are reloaded only when
// the column enters a new coarse layer. The 3D FP32 form is held to 64 registers, so that the
// 8 blocks per CU of a 256 x 256 x 128 grid are resident at once. SR: single resolution (the
// phase field on the flow grid; the face velocities are taken as they are).
template <typename T, int R, int MODE, bool RELAX, int TXC = 0, bool MOVE = false>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && R == 2 && MODE == 0 && !RELAX ? 8
                                       : (RELAX && sizeof(T) == 8 ? 3 : 4))))
    k_ch_rhs(const T* __restrict__ phin, const T* __restrict__ phinm1, Prolonged<T> pv,
             T* __restrict__ out, const T* __restrict__ advp, int nx, int ny, int nz, int KB, T ihx,
             T ihy, T ihz, StepConsts c) {
  extern __shared__ __align__(16) unsigned char smem[];
  // TXC > 0: the block shape TXC x 4 known at compile time (LDS neighbours at immediate offsets)
  const int TX = TXC > 0 ? TXC : (int)blockDim.x, TY = TXC > 0 ? 4 : (int)blockDim.y;
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
  const size_t layer = (size_t)ny * nx;
  // tile points of this thread (own_first_point: point 0 is the thread's own column) and
  // their in-layer byte offsets: the loads take a uniform layer base plus a 32-bit lane offset
  unsigned hOff[R];
  int hE[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    int hy = 0, hx = 0;
    hE[q] = own_first_point<1, 1>(TX, TY, tid, q, hy, hx) ? hy * HX + hx : HP;
    hOff[q] = hE[q] < HP ? (unsigned)(wrap(Y0 - 1 + hy, ny) * nx + wrap(X0 - 1 + hx, nx)) * sizeof(T) : 0u;
  }
  auto has = [&](int q) { return hE[q] < HP; };
  // beyond a wall the zero-flux ghost is the adjacent layer
  auto kcl = [&](int Kl) { return min(max(Kl, 0), nz - 1); };
  auto load_tile = [&](int Kl, T* a, T* b) {
    const T* pa = phin + kcl(Kl) * layer;
    const T* pb = phinm1 + kcl(Kl) * layer;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (has(q)) {
        a[q] = ld_at(pa, hOff[q]);
        if (!first) b[q] = ld_at(pb, hOff[q]);
      }
    }
  };
  auto store_tile = [&](int slot, const T* a, const T* b) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (has(q)) {
        const T p = first ? a[q] : (T)2 * a[q] - b[q];
        sP[slot * HP + hE[q]] = p;
        sW[slot * HP + hE[q]] = (p * p * p - p) * icn2 - sc * p;
      }
    }
  };
  const unsigned cid = (J * nx + I) * sizeof(T);
  // phi_hat of the layer whose tile a, b hold (point 0: the thread's own column)
  auto own_hat = [&](const T* a, const T* b) -> T { return first ? a[0] : (T)2 * a[0] - (T)0.5 * b[0]; };
  // coarse column of this fine column (eq. dual1); with a single resolution the column itself
  const int ry = pv.ry;
  constexpr bool sr = MODE == 1;   // single resolution (pv.single)
  constexpr bool pre = MODE == 2;  // advection given (WENO-Z), no velocities needed
  const bool vy = pv.cny > 1;
  const int ic = sr ? I : (I >> 1), icw = wrap(ic - 1, pv.cnx);
  const int jc = ry == 2 ? (J >> 1) : J, jcw = vy ? wrap(jc - 1, pv.cny) : 0;
  const int cplane = pv.cnx * pv.cny;
  const int cu0 = jc * pv.cnx + ic, cu1 = jc * pv.cnx + icw;
  const int cv1 = jcw * pv.cnx + ic;
  // raw coarse values of one coarse layer: u at cu0, cu1; v at cu0, cv1; w at k and k - 1,
  // each at levels n and n - 1
  auto load_vel = [&](int k, T* vn, T* vm) {
    const int o = k * cplane;
    vn[0] = pv.un[o + cu0];
    vn[1] = pv.un[o + cu1];
    vn[2] = pv.vn[o + cu0];
    vn[3] = vy ? pv.vn[o + cv1] : (T)0;
    vn[4] = k < pv.cnz - 1 ? pv.wn[o + cu0] : (T)0;
    vn[5] = k > 0 ? pv.wn[o - cplane + cu0] : (T)0;
    if (!first) {
      vm[0] = pv.unm1[o + cu0];
      vm[1] = pv.unm1[o + cu1];
      vm[2] = pv.vnm1[o + cu0];
      vm[3] = vy ? pv.vnm1[o + cv1] : (T)0;
      vm[4] = k < pv.cnz - 1 ? pv.wnm1[o + cu0] : (T)0;
      vm[5] = k > 0 ? pv.wnm1[o - cplane + cu0] : (T)0;
    }
  };
  const T ihx2 = ihx * ihx, ihy2 = ihy * ihy, ihz2 = ihz * ihz, h = (T)0.5;
  const T gb = (T)c.g_bot * ihz, gt = (T)c.g_top * ihz;
  constexpr bool relax = RELAX;  // relaxed walls (eq. NS34 with D_w > 0)
  const T kg = RELAX ? (T)(c.relax_kappa * c.inv_gamma0) * ihz : (T)0;
  auto phat_at = [&](int Kl, int Jl, int Il) -> T {
    const size_t id = ((size_t)Kl * ny + wrap(Jl, ny)) * nx + wrap(Il, nx);
    return first ? phin[id] : (T)2 * phin[id] - (T)0.5 * phinm1[id];
  };
  // relaxed moving walls (MOVE, eq. NS34): the wall advection D_w u_w . grad phi* of the
  // right-hand side enters the ghost as phi_hat - dt u_w . grad phi* in place of phi_hat
  // (kappa dt / gamma0 = D_w), u_w the wall's own velocity (eq. NS13), the in-plane derivatives
  // of phi* central on the wall-adjacent layer. An instantiation of its own: the extra loads
  // would cost the static-wall forms registers.
  auto pstar_at = [&](int Kl, int Jl, int Il) -> T {
    const size_t id = ((size_t)Kl * ny + wrap(Jl, ny)) * nx + wrap(Il, nx);
    return first ? phin[id] : (T)2 * phin[id] - phinm1[id];
  };
  auto phat_wall = [&](int Kl, int Jl, int Il) -> T {
    T ph = phat_at(Kl, Jl, Il);
    if constexpr (MOVE) {
      const double* uw = Kl == 0 ? c.uwb : c.uwt;
      const T adv = (T)uw[0] * (pstar_at(Kl, Jl, Il + 1) - pstar_at(Kl, Jl, Il - 1)) * ((T)0.5 * ihx) +
                    (T)uw[1] * (pstar_at(Kl, Jl + 1, Il) - pstar_at(Kl, Jl - 1, Il)) * ((T)0.5 * ihy);
      ph -= (T)c.dt * adv;
    }
    return ph;
  };
  T ta[R], tb[R];
  int sm = 0, s0 = 1, sp = 2;
  load_tile(K0 - 1, ta, tb);
  store_tile(sm, ta, tb);
  load_tile(K0, ta, tb);
  store_tile(s0, ta, tb);
  T phat_next = own_hat(ta, tb);
  load_tile(K0 + 1, ta, tb);
  T ufp = 0, ufm = 0, vfp = 0, vfm = 0, wk = 0, wkm = 0;
  int kcur = -1;
  for (int K = K0; K < K0 + KB; ++K) {
    const int k = sr ? K : (K >> 1);
    if (!pre && k != kcur) {
      kcur = k;
      T vn[6], vm[6], s[6];
      load_vel(k, vn, vm);
#pragma unroll
      for (int m = 0; m < 6; ++m) s[m] = first ? vn[m] : (T)2 * vn[m] - vm[m];
      if (sr) {
        ufp = s[0];
        ufm = s[1];
      } else {
        const bool iodd = I & 1;
        ufp = iodd ? s[0] : h * (s[1] + s[0]);
        ufm = iodd ? h * (s[1] + s[0]) : s[1];
      }
      if (ry == 2) {
        const bool jodd = J & 1;
        vfp = jodd ? s[2] : h * (s[3] + s[2]);
        vfm = jodd ? h * (s[3] + s[2]) : s[3];
      } else if (vy) {
        vfp = s[2];
        vfm = s[3];
      } else {
        vfp = vfm = s[2];
      }
      wk = s[4];
      wkm = s[5];
    }
    const T phat = phat_next;
    // layer K + 1 enters the ring; the layer after it and the next centre values go out
    store_tile(sp, ta, tb);
    if (K + 1 < K0 + KB) {
      phat_next = own_hat(ta, tb);
      load_tile(K + 2, ta, tb);
    }
    // fine z faces K (above) and K-1 (below); the walls carry zero flux
    const T wfp = K == nz - 1 ? (T)0 : (sr || (K & 1) ? wk : h * (wkm + wk));
    const T wfm = K == 0 ? (T)0 : (sr ? wkm : ((K & 1) ? h * (wkm + wk) : wkm));
    __syncthreads();
    const int c0 = (ty + 1) * HX + (tx + 1);
    const T* P0 = sP + s0 * HP;
    const T* W0 = sW + s0 * HP;
    const T p0 = P0[c0], pxp = P0[c0 + 1], pxm = P0[c0 - 1], pyp = P0[c0 + HX], pym = P0[c0 - HX];
    const T pzp = sP[sp * HP + c0], pzm = sP[sm * HP + c0];
    const T w0 = W0[c0];
    const T lapw = (W0[c0 + 1] - 2 * w0 + W0[c0 - 1]) * ihx2 + (W0[c0 + HX] - 2 * w0 + W0[c0 - HX]) * ihy2 +
                   (sW[sp * HP + c0] - 2 * w0 + sW[sm * HP + c0]) * ihz2;
    const T adv = pre ? ld_at(advp + K * layer, cid) :
                        (ufp * h * (p0 + pxp) - ufm * h * (pxm + p0)) * ihx +
                  (vfp * h * (p0 + pyp) - vfm * h * (pym + p0)) * ihy +
                  (wfp * h * (p0 + pzp) - wfm * h * (pzm + p0)) * ihz;
    // wetting data b = g(phi*) / hz on the wall-adjacent layers, and L_N b; relaxed walls
    // (eq. NS34, D_w > 0) add (kappa / hz) phi_hat / gamma0 to it, phi_hat read on those
    // layers only
    auto bval = [&](int kk, T p, T ph) -> T {
      T b = 0;
      if (kk == 0) b += gb * ((T)1 - p * p);
      if (kk == nz - 1) b += gt * ((T)1 - p * p);
      if (RELAX && (kk == 0 || kk == nz - 1)) b += kg * ph;
      return b;
    };
    T lapb = 0;
    if (K == 0 || K == nz - 1) {
      const T b0 = bval(K, p0, relax ? phat_wall(K, J, I) : (T)0);
      lapb = (bval(K, pxp, relax ? phat_wall(K, J, I + 1) : (T)0) - 2 * b0 +
              bval(K, pxm, relax ? phat_wall(K, J, I - 1) : (T)0)) * ihx2 +
             (bval(K, pyp, relax ? phat_wall(K, J + 1, I) : (T)0) - 2 * b0 +
              bval(K, pym, relax ? phat_wall(K, J - 1, I) : (T)0)) * ihy2;
      const T bup = K + 1 < nz ? bval(K + 1, pzp, (T)0) : b0;
      const T bdn = K > 0 ? bval(K - 1, pzm, (T)0) : b0;
      lapb += (bup - 2 * b0 + bdn) * ihz2;
    } else {
      if (K == 1) lapb += bval(0, pzm, relax ? phat_wall(0, J, I) : (T)0) * ihz2;
      if (K == nz - 2) lapb += bval(nz - 1, pzp, relax ? phat_wall(nz - 1, J, I) : (T)0) * ihz2;
    }
    const T q = (T)c.pe_cn2 * (phat * (T)c.inv_dt - adv) + lapw;
    st_at(out + K * layer, cid, q - lapb);
    __syncthreads();
    const int t = sm;
    sm = s0;
    s0 = sp;
    sp = t;
  }
}


// Chemical potential, restriction and properties, z-marching: a block owns CX x CY coarse
// columns and KB coarse layers. A ring of four fine layers of phi^{n+1} (one-cell halo) and a
// ring of three fine layers of G live in LDS, indexed by the clamped fine layer modulo the
// ring size; stepping one coarse layer up replaces two phi layers and evaluates G on two new
// layers. The block has 2 CY rows of threads: all of them load tiles and evaluate G; for the
// restricted sums the lower CY rows form the phi-derived outputs and the upper CY rows the
// G-derived ones of the same coarse cells. Each thread owns at most R points of a tile (their
// in-layer offsets are computed once); the global loads of the layers that the next step
// needs are issued one step ahead into registers, so that they are in flight while the
// block evaluates G and forms the next sums. The FP32 form of the common case is held to six
// wavefronts per SIMD (80 registers, a few spilled): at 256 x 256 x 128 coarse cells that makes
// one round of six blocks per CU with marches of 43 layers, measured 15% faster than five
// wavefronts (one round of four blocks, marches of 64).
template <typename T, int R, bool RELAX, int CXC = 0, bool MOVE = false>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && R == 3 && !RELAX ? 6 : 1)))
    k_restrict_g(const T* __restrict__ phinew, const T* __restrict__ phin,
                 const T* __restrict__ phinm1, Restricted<T> r, int fnx, int fny, int fnz,
                 T fihx, T fihy, T fihz, int cnx, int cny, int cnz, int ry, int KB,
                 StepConsts c) {
  extern __shared__ __align__(16) unsigned char smem[];
  // CXC > 0: the block shape CXC x (256 / 2 CXC) coarse columns known at compile time
  const int CX = CXC > 0 ? CXC : (int)blockDim.x, CY = CXC > 0 ? kBlock / (2 * CXC) : (int)blockDim.y / 2;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i0 = bx * CX, j0 = by * CY, k0 = bz * KB;
  const int k1 = min(k0 + KB, cnz);  // the last block of a column may march fewer layers
  const int GX = 2 * CX + 1, GY = ry * CY + 1, GP = GX * GY;
  const int PX = GX + 2, PY = GY + 2, PP = PX * PY;
  const int X0 = 2 * i0, Y0 = ry * j0;
  const int tid = threadIdx.y * CX + threadIdx.x;
  const int nth = CX * blockDim.y;
  // rings of 4 phi slots (PP entries) and 3 G slots (GP entries), then a scratch area of
  // R nth - GP entries: the points past a tile are computed and stored there, so that no tile
  // loop branches
  T* sP = reinterpret_cast<T*>(smem);
  T* sG = sP + 4 * PP;
  T* sX = sG + 3 * GP;
  const bool first = c.first != 0;
  const T ihx2 = fihx * fihx, ihy2 = fihy * fihy, ihz2 = fihz * fihz;
  const T cn2 = (T)c.cn2, S = (T)c.S;
  const T gb = (T)c.g_bot * fihz, gt = (T)c.g_top * fihz;
  constexpr bool relax = RELAX;  // relaxed walls (eq. NS34 with D_w > 0)
  const T kk = RELAX ? (T)c.relax_kappa * fihz : (T)0;
  const T kg = RELAX ? (T)(c.relax_kappa * c.inv_gamma0) * fihz : (T)0;
  const size_t layer = (size_t)fny * fnx;
  auto kc = [&](int Kf) { return min(max(Kf, 0), fnz - 1); };
  // per-thread tile points: in-layer byte offsets of the phi tile (with halo) and of the G
  // tile (a uniform layer base plus a 32-bit lane offset), and the LDS index of each G point
  // in the phi tile. Points past a tile read the layer's first element and an interior LDS
  // point.
  unsigned pOff[R], gOff[R];
  int gM[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int e = tid + q * nth;
    const int py = e / PX, px = e - py * PX;
    const int gy = e / GX, gx = e - gy * GX;
    pOff[q] = e < PP ? (unsigned)(wrap(Y0 - 1 + py, fny) * fnx + wrap(X0 - 1 + px, fnx)) * sizeof(T) : 0u;
    gOff[q] = e < GP ? (unsigned)(wrap(Y0 + gy, fny) * fnx + wrap(X0 + gx, fnx)) * sizeof(T) : 0u;
    gM[q] = e < GP ? (gy + 1) * PX + gx + 1 : PX + 1;
  }
  auto load_p = [&](int Kf, T* v) {
    const T* src = phinew + kc(Kf) * layer;
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = ld_at(src, pOff[q]);
  };
  auto store_p = [&](int Kf, const T* v) {
    T* dst = sP + (kc(Kf) & 3) * PP;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = tid + q * nth;
      *(e < PP ? dst + e : sX + (e - PP)) = v[q];
    }
  };
  // phi* at the G points of fine layer Kf
  auto load_ps = [&](int Kf, T* v) {
    const T* a = phin + kc(Kf) * layer;
    const T* b = phinm1 + kc(Kf) * layer;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const T an = ld_at(a, gOff[q]);
      v[q] = first ? an : (T)2 * an - ld_at(b, gOff[q]);
    }
  };
  // G on fine layer Kf from the phi ring and phi* at the G points
  auto compute_g = [&](int Kf, const T* psr) {
    const int K = kc(Kf);
    const T* Pm = sP + (kc(K - 1) & 3) * PP;
    const T* P0 = sP + (K & 3) * PP;
    const T* Pp = sP + (kc(K + 1) & 3) * PP;
    T* dst = sG + (K % 3) * GP;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      {
        const int e = tid + q * nth;
        const int m = gM[q];
        const T p = P0[m];
        const T lap = (P0[m + 1] - 2 * p + P0[m - 1]) * ihx2 + (P0[m + PX] - 2 * p + P0[m - PX]) * ihy2 +
                      (Pp[m] - 2 * p + Pm[m]) * ihz2;
        const T ps = psr[q];
        T b = 0;
        if (K == 0) b += gb * ((T)1 - ps * ps);
        if (K == fnz - 1) b += gt * ((T)1 - ps * ps);
        if (relax && (K == 0 || K == fnz - 1)) {
          // relaxed walls: (kappa / hz)(phi_hat / gamma0 - phi^{n+1}) in the wall ghost
          const T an = ld_at(phin + K * layer, gOff[q]);
          T ph = first ? an : (T)2 * an - (T)0.5 * ld_at(phinm1 + K * layer, gOff[q]);
          if constexpr (MOVE) {
            // moving walls: phi_hat - dt u_w . grad phi* (eq. NS34), as in the right-hand side
            const int idx = (int)(gOff[q] / sizeof(T)), I = idx % fnx, J = idx / fnx;
            const T* a = phin + K * layer;
            const T* b1 = phinm1 + K * layer;
            auto pst = [&](int jj, int ii) {
              const int o = wrap(jj, fny) * fnx + wrap(ii, fnx);
              return first ? a[o] : (T)2 * a[o] - b1[o];
            };
            const double* uw = K == 0 ? c.uwb : c.uwt;
            const T adv = (T)uw[0] * (pst(J, I + 1) - pst(J, I - 1)) * ((T)0.5 * fihx) +
                          (T)uw[1] * (pst(J + 1, I) - pst(J - 1, I)) * ((T)0.5 * fihy);
            ph -= (T)c.dt * adv;
          }
          b += kg * ph - kk * p;
        }
        *(e < GP ? dst + e : sX + (e - GP)) = -cn2 * (lap + b) + S * (p - ps) + ps * ps * ps - ps;
      }
    }
  };
  // registers in flight: phi on the two fine layers and phi* on the two G layers that the
  // next step brings in
  T pfa[R], pfb[R], psa[R], psb[R];
  {
    // G on fine layers 2k0 .. 2k0+2 needs phi on 2k0-1 .. 2k0+3; with a ring of four the
    // layer 2k0+3 enters after G on 2k0 and 2k0+1 (its slot is that of 2k0-1)
    T ps0[R], ps1[R];
    load_p(2 * k0 - 1, pfa);
    load_p(2 * k0, pfb);
    load_ps(2 * k0, ps0);
    load_ps(2 * k0 + 1, ps1);
    store_p(2 * k0 - 1, pfa);
    store_p(2 * k0, pfb);
    load_p(2 * k0 + 1, pfa);
    load_p(2 * k0 + 2, pfb);
    store_p(2 * k0 + 1, pfa);
    store_p(2 * k0 + 2, pfb);
    load_p(2 * k0 + 3, pfa);
    __syncthreads();
    compute_g(2 * k0, ps0);
    compute_g(2 * k0 + 1, ps1);
    load_ps(2 * k0 + 2, ps0);
    __syncthreads();
    store_p(2 * k0 + 3, pfa);
    __syncthreads();
    compute_g(2 * k0 + 2, ps0);
    __syncthreads();
    if (k1 - k0 > 1) {
      load_p(2 * k0 + 4, pfa);
      load_p(2 * k0 + 5, pfb);
      load_ps(2 * k0 + 3, psa);
      load_ps(2 * k0 + 4, psb);
    }
  }
  const int tx = threadIdx.x;
  const bool upper = (int)threadIdx.y >= CY;
  const int ty = upper ? threadIdx.y - CY : threadIdx.y;
  const int i = i0 + tx, j = j0 + ty;
  const T r1 = (T)c.rho1, r2 = (T)c.rho2, m1 = (T)c.mu1, m2 = (T)c.mu2, hf = (T)0.5;
  auto rinv = [&](T ph) { return (T)1 / (hf * ((T)1 + ph) * r1 + hf * ((T)1 - ph) * r2); };
  auto mu = [&](T ph) { return hf * ((T)1 + ph) * m1 + hf * ((T)1 - ph) * m2; };
  const int plane = cnx * cny;
  const int ndy = ry + 1;
  for (int k = k0; k < k1; ++k) {
    // Separable sums of the tensor-product rule: per z layer and y row, x sums over the
    // centre pair (dx 0,1) and the face pair (dx 1,2); then y pairs, then z pairs. The 1/8
    // weight is applied once at the end (a centre-located y axis without refinement counts
    // its single cell twice). Lower rows: phi (ring of 4); upper rows: G (ring of 3).
    {
      T z_[3][4];  // per dz: [YcXc, YcXf, YfXc, YfXf]
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const int K = kc(2 * k + dz);
        T xc[3], xf[3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int gy = ry * ty + (dy < ndy ? dy : 0);
          const T* pr = upper ? sG + (K % 3) * GP + gy * GX + 2 * tx
                              : sP + (K & 3) * PP + (gy + 1) * PX + 2 * tx + 1;
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
    if (k + 1 < k1) {
      // phi on 2k+4, 2k+5 replaces 2k, 2k+1 (no longer read); G on 2k+3, 2k+4 replaces
      // 2k, 2k+1. The loads for the step after next go out before G is evaluated.
      __syncthreads();
      store_p(2 * k + 4, pfa);
      store_p(2 * k + 5, pfb);
      T p3[R], p4[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        p3[q] = psa[q];
        p4[q] = psb[q];
      }
      if (k + 2 < k1) {
        load_p(2 * k + 6, pfa);
        load_p(2 * k + 7, pfb);
        load_ps(2 * k + 5, psa);
        load_ps(2 * k + 6, psb);
      }
      __syncthreads();
      compute_g(2 * k + 3, p3);
      compute_g(2 * k + 4, p4);
      __syncthreads();
    }
  }
}
// div(u_f phi*) on the fine grid with WENO-Z face values (the advection of eq. NS25), phi* =
// 2 phi^n - phi^{n-1} (phi^n on the first step), face velocities prolonged on the fly (eq.
// dual1; as they are at a single resolution). A z-march that evaluates every face once: a
// block owns TX x TY fine columns and KB layers; phi* of the current layer with a three-cell
// halo sits in LDS, each thread keeps phi* of its column from K-4 to K+3 in registers (z
// mirrored at the walls), the x- and y-face fluxes of the layer go to LDS (faces spread over
// the threads, the x overhang on the first wave and the y overhang on the second), and the z
// flux through the top face becomes the next layer's bottom flux. Y3D = false: the 2D form
// (one cell in y, no y flux).
template <typename T, bool Y3D>
__global__ void __launch_bounds__(256)
    k_weno_adv_zm(const T* __restrict__ phin, const T* __restrict__ phinm1, Prolonged<T> pv,
                  T* __restrict__ adv, int nx, int ny, int nz, int KB, T ihx, T ihy, T ihz) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TX = blockDim.x, TY = blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int X0 = bx * TX, Y0 = by * TY, K0 = bz * KB;
  const int K1 = min(K0 + KB, nz);
  const int HX = TX + 6, HY = Y3D ? TY + 6 : 1, HP = HX * HY;
  T* sT = reinterpret_cast<T*>(smem);  // phi* of the layer [HY][HX]
  T* sFx = sT + HP;                     // x-face fluxes [TY][TX + 1]
  T* sFy = sFx + TY * (TX + 1);         // y-face fluxes [TY + 1][TX]
  const int tx = threadIdx.x, ty = threadIdx.y, nth = TX * TY;
  const int tid = ty * TX + tx;
  const int I = X0 + tx, J = Y0 + ty;
  const bool first = pv.first != 0;
  const size_t layer = (size_t)ny * nx;
  auto ps_at = [&](int Kl, int off) -> T {
    const size_t id = (size_t)Kl * layer + off;
    return first ? phin[id] : (T)2 * phin[id] - phinm1[id];
  };
  const int col = J * nx + I;
  T zw[8];  // phi* at K-4 .. K+3 of this column
#pragma unroll
  for (int d = 0; d < 8; ++d) zw[d] = ps_at(mirror_index(K0 - 4 + d, nz), col);
  T fbot = weno_flux(pv.wf(K0 - 1, J, I), zw[1], zw[2], zw[3], zw[4], zw[5], zw[6]);
  // this thread's tile points and faces, the same on every layer: decomposed once (at most
  // NT tile points and two faces of each direction per thread; checked by the launcher)
  constexpr int NT = Y3D ? 4 : 2;
  const int nfx = (TX + 1) * TY, nfy = TX * (TY + 1);
  int tOff[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const int e = tid + q * nth;
    const int hy = e / HX, hx = e - hy * HX;
    tOff[q] = e < HP ? (Y3D ? wrap(Y0 - 3 + hy, ny) : 0) * nx + wrap(X0 - 3 + hx, nx) : -1;
  }
  int xr[2], xc[2], yr[2], yc[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int f = tid + q * nth;
    xr[q] = f < nfx ? f / (TX + 1) : -1;
    xc[q] = f < nfx ? f - xr[q] * (TX + 1) : 0;
    // the y faces rotated by one wave, so that their overhang lands on another wave than x's
    const int g = (f + 64) % nfy;
    yr[q] = f < nfy ? g / TX : -1;
    yc[q] = f < nfy ? g - yr[q] * TX : 0;
  }
  // the tile of the next layer is loaded while the current one is evaluated
  T pa[NT], pb[NT];
  auto load_tile = [&](int Kl) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      if (tOff[q] >= 0) {
        const size_t id = (size_t)Kl * layer + tOff[q];
        pa[q] = phin[id];
        if (!first) pb[q] = phinm1[id];
      }
    }
  };
  load_tile(K0);
  // x and y face velocities of the thread's faces: constant over the two fine layers of a
  // coarse layer (dual resolution), so formed when the coarse layer changes
  T xu[2] = {0, 0}, yv[2] = {0, 0};
  for (int K = K0; K < K1; ++K) {
#pragma unroll
    for (int q = 0; q < NT; ++q)
      if (tOff[q] >= 0) sT[tid + q * nth] = first ? pa[q] : (T)2 * pa[q] - pb[q];
    if (K + 1 < K1) load_tile(K + 1);
    if (pv.single || K == K0 || (K & 1) == 0) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (xr[q] >= 0) xu[q] = pv.uf(K, Y0 + xr[q], X0 - 1 + xc[q]);
        if (Y3D && yr[q] >= 0) yv[q] = pv.vf(K, Y0 - 1 + yr[q], X0 + yc[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (xr[q] >= 0) {
        const int r = xr[q], c = xc[q];
        const T* v = sT + (Y3D ? r + 3 : 0) * HX + c;  // cells X0 - 3 + c .. X0 + 2 + c
        sFx[r * (TX + 1) + c] = weno_flux(xu[q], v[0], v[1], v[2], v[3], v[4], v[5]);
      }
    }
    if (Y3D) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (yr[q] >= 0) {
          const int r = yr[q], c = yc[q];
          const T* v = sT + r * HX + c + 3;  // rows Y0 - 3 + r .. Y0 + 2 + r
          sFy[r * TX + c] = weno_flux(yv[q], v[0], v[HX], v[2 * HX], v[3 * HX], v[4 * HX], v[5 * HX]);
        }
      }
    }
    const T ftop = weno_flux(pv.wf(K, J, I), zw[2], zw[3], zw[4], zw[5], zw[6], zw[7]);
    __syncthreads();
    T d = (sFx[ty * (TX + 1) + tx + 1] - sFx[ty * (TX + 1) + tx]) * ihx + (ftop - fbot) * ihz;
    if (Y3D) d += (sFy[(ty + 1) * TX + tx] - sFy[ty * TX + tx]) * ihy;
    adv[(size_t)K * layer + col] = d;
    fbot = ftop;
#pragma unroll
    for (int q = 0; q < 7; ++q) zw[q] = zw[q + 1];
    if (K + 1 < K1) zw[7] = ps_at(mirror_index(K + 4, nz), col);
  }
}

// Single resolution (the phase field on the flow grid): chemical potential G^{n+1} (the
// bracket of eq. NS25 times the mixing energy, as restrict_g) and phi at the cells.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_g_single(const T* __restrict__ phinew, const T* __restrict__ phin,
               const T* __restrict__ phinm1, Restricted<T> r, int nx, int ny, int nz, T ihx, T ihy,
               T ihz, StepConsts c) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x, j = by * blockDim.y + threadIdx.y, k = bz;
  const int id = (k * ny + j) * nx + i;
  auto at = [&](int kk, int jj, int ii) {
    return phinew[(min(max(kk, 0), nz - 1) * ny + wrap(jj, ny)) * nx + wrap(ii, nx)];
  };
  const T p = phinew[id];
  const T lap = (at(k, j, i + 1) - 2 * p + at(k, j, i - 1)) * (ihx * ihx) +
                (at(k, j + 1, i) - 2 * p + at(k, j - 1, i)) * (ihy * ihy) +
                (at(k + 1, j, i) - 2 * p + at(k - 1, j, i)) * (ihz * ihz);
  const T an = phin[id];
  const T ps = c.first ? an : (T)2 * an - phinm1[id];
  T b = 0;
  if (k == 0) b += (T)c.g_bot * ihz * ((T)1 - ps * ps);
  if (k == nz - 1) b += (T)c.g_top * ihz * ((T)1 - ps * ps);
  if (c.relax_kappa != 0.0 && (k == 0 || k == nz - 1)) {
    // relaxed walls: (kappa / hz)(phi_hat / gamma0 - phi^{n+1}) in the wall ghost; moving
    // walls: phi_hat - dt u_w . grad phi* (eq. NS34)
    T ph = c.first ? an : (T)2 * an - (T)0.5 * phinm1[id];
    const double* uw = k == 0 ? c.uwb : c.uwt;
    if (uw[0] != 0.0 || uw[1] != 0.0) {
      auto pst = [&](int jj, int ii) {
        const int o = (k * ny + wrap(jj, ny)) * nx + wrap(ii, nx);
        return c.first ? phin[o] : (T)2 * phin[o] - phinm1[o];
      };
      const T adv = (T)uw[0] * (pst(j, i + 1) - pst(j, i - 1)) * ((T)0.5 * ihx) +
                    (T)uw[1] * (pst(j + 1, i) - pst(j - 1, i)) * ((T)0.5 * ihy);
      ph -= (T)c.dt * adv;
    }
    b += (T)(c.relax_kappa * c.inv_gamma0) * ihz * ph - (T)c.relax_kappa * ihz * p;
  }
  r.G_c[id] = -(T)c.cn2 * (lap + b) + (T)c.S * (p - ps) + ps * ps * ps - ps;
  r.phi_c[id] = p;
}

// Single resolution: the face and edge quantities of the restricted set from the cell
// values (eq. dual2's rule without refinement: a face is the mean of its two cells, an edge
// the mean of its four, each as a mean along x, then y, then z; the wall ghost is the
// adjacent cell) and the mixture properties of eq. dual3.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_props_single(Restricted<T> r, int nx, int ny, int nz, StepConsts c) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x, j = by * blockDim.y + threadIdx.y, k = bz;
  const int id = (k * ny + j) * nx + i;
  const int plane = nx * ny;
  auto P = [&](int kk, int jj, int ii) { return r.phi_c[(min(max(kk, 0), nz - 1) * ny + wrap(jj, ny)) * nx + wrap(ii, nx)]; };
  auto Gv = [&](int kk, int jj, int ii) { return r.G_c[(min(max(kk, 0), nz - 1) * ny + wrap(jj, ny)) * nx + wrap(ii, nx)]; };
  const T h = (T)0.5;
  const T r1 = (T)c.rho1, r2 = (T)c.rho2, m1 = (T)c.mu1, m2 = (T)c.mu2;
  auto rinv = [&](T ph) { return (T)1 / (h * ((T)1 + ph) * r1 + h * ((T)1 - ph) * r2); };
  auto mu = [&](T ph) { return h * ((T)1 + ph) * m1 + h * ((T)1 - ph) * m2; };
  const T p0 = P(k, j, i);
  r.G_x[id] = h * (Gv(k, j, i) + Gv(k, j, i + 1));
  r.G_y[id] = h * (Gv(k, j, i) + Gv(k, j + 1, i));
  r.G_z[id] = h * (Gv(k, j, i) + Gv(k + 1, j, i));
  r.ri_x[id] = rinv(h * (p0 + P(k, j, i + 1)));
  r.ri_y[id] = rinv(h * (p0 + P(k, j + 1, i)));
  r.ri_z[id] = rinv(h * (p0 + P(k + 1, j, i)));
  r.mu_c[id] = mu(p0);
  r.mu_xy[id] = mu(h * (h * (p0 + P(k, j, i + 1)) + h * (P(k, j + 1, i) + P(k, j + 1, i + 1))));
  // z-edge arrays carry nz + 1 layers: layer m is the edge at z = m hz
  auto exz = [&](int m) { return mu(h * (h * (P(m - 1, j, i) + P(m - 1, j, i + 1)) + h * (P(m, j, i) + P(m, j, i + 1)))); };
  auto eyz = [&](int m) { return mu(h * (h * (P(m - 1, j, i) + P(m - 1, j + 1, i)) + h * (P(m, j, i) + P(m, j + 1, i)))); };
  r.mu_xz[id + plane] = exz(k + 1);
  r.mu_yz[id + plane] = eyz(k + 1);
  if (k == 0) {
    r.mu_xz[id] = exz(0);
    r.mu_yz[id] = eyz(0);
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
  const int single = f.nx == c.nx ? 1 : 0;  // the phase field on the flow grid
  Prolonged<T> pv{in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1, c.nx, c.ny, c.nz,
                  (c.ny == 1 || single) ? 1 : 2, k.first, single};
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
  const int HP = (TX + 2) * (TY + 2);
  const int need = (HP + TX * TY - 1) / (TX * TY);
  if (need > 4) return hipErrorInvalidConfiguration;
  const size_t shm = (size_t)6 * HP * sizeof(T);
  const dim3 grid(f.nx / TX, f.ny / TY, f.nz / KB), block(TX, TY, 1);
#define DRPF_CH(R, MODE, RELAX, TXC, ...)                                                          \
  hipLaunchKernelGGL((k_ch_rhs<T, R, MODE, RELAX, TXC, ##__VA_ARGS__>), grid, block, shm, st, in.phin, \
                     in.phinm1, pv, rhs, in.adv, f.nx, f.ny, f.nz, KB, (T)f.ihx, (T)f.ihy, (T)f.ihz, k)
  // the 64 x 4 tile of 3D grids with its shape at compile time
  const bool t64 = TX == 64 && TY == 4;
#define DRPF_CH_R(MODE, RELAX)      \
  if (t64)                          \
    DRPF_CH(2, MODE, RELAX, 64);    \
  else if (need <= 2)               \
    DRPF_CH(2, MODE, RELAX, 0);     \
  else                              \
    DRPF_CH(4, MODE, RELAX, 0)
  // mode: 0 dual resolution, 1 single resolution, 2 advection given
  const int mode = in.adv ? 2 : (single ? 1 : 0);
  const bool moving = k.uwb[0] != 0.0 || k.uwb[1] != 0.0 || k.uwt[0] != 0.0 || k.uwt[1] != 0.0;
#define DRPF_CH_M(MODE)                  \
  if (need <= 2)                         \
    DRPF_CH(2, MODE, true, 0, true);     \
  else                                   \
    DRPF_CH(4, MODE, true, 0, true)
  if (k.relax_kappa != 0.0 && moving) {
    if (mode == 2) { DRPF_CH_M(2); } else if (mode == 1) { DRPF_CH_M(1); } else { DRPF_CH_M(0); }
  } else if (k.relax_kappa != 0.0) {
    if (mode == 2) { DRPF_CH_R(2, true); } else if (mode == 1) { DRPF_CH_R(1, true); } else { DRPF_CH_R(0, true); }
  } else {
    if (mode == 2) { DRPF_CH_R(2, false); } else if (mode == 1) { DRPF_CH_R(1, false); } else { DRPF_CH_R(0, false); }
  }
#undef DRPF_CH_M
#undef DRPF_CH_R
#undef DRPF_CH
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
  const int GX = 2 * CX + 1, GY = ry * CY + 1;
  const int PP = (GX + 2) * (GY + 2), nth = 2 * CX * CY;
  // each thread keeps at most R points of a tile in registers
  const int need = (PP + nth - 1) / nth;
  if (need > 6) return hipErrorInvalidConfiguration;
  const int GP = GX * GY, Rk = need <= 3 ? 3 : 6;
  const size_t shm = (size_t)(4 * PP + 3 * GP + Rk * nth - GP) * sizeof(T);
  const int cols = (c.nx / CX) * (c.ny / CY);
  const dim3 block(CX, 2 * CY, 1);
  // coarse layers per block: the march amortises the fine z halo; one round of blocks
  auto go = [&](auto kernel) {
    const int KB = march_layers(kernel, nth, shm, cols, c.nz);
    const dim3 grid(c.nx / CX, c.ny / CY, (c.nz + KB - 1) / KB);
    hipLaunchKernelGGL(kernel, grid, block, shm, st, phinew, phin, phinm1, r, f.nx, f.ny, f.nz, (T)f.ihx,
                       (T)f.ihy, (T)f.ihz, c.nx, c.ny, c.nz, ry, KB, k);
  };
  const bool moving = k.uwb[0] != 0.0 || k.uwb[1] != 0.0 || k.uwt[0] != 0.0 || k.uwt[1] != 0.0;
  if (k.relax_kappa != 0.0 && moving) {
    if (Rk == 3) go(k_restrict_g<T, 3, true, 0, true>); else go(k_restrict_g<T, 6, true, 0, true>);
  } else if (k.relax_kappa != 0.0) {
    if (Rk == 3) go(k_restrict_g<T, 3, true>); else go(k_restrict_g<T, 6, true>);
  } else {
    if (CX == 32 && CY == 4) go(k_restrict_g<T, 3, false, 32>);
    else if (Rk == 3) go(k_restrict_g<T, 3, false>);
    else go(k_restrict_g<T, 6, false>);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_weno_adv_fine(const Dims& f, const Dims& c, const StepConsts& k, ChIn<T> in, T* adv,
                                hipStream_t st) {
  const int single = f.nx == c.nx ? 1 : 0;
  Prolonged<T> pv{in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1, c.nx, c.ny, c.nz,
                  (c.ny == 1 || single) ? 1 : 2, k.first, single};
  // z-march: 64 x 4 columns (2D: up to 256 x 1), KB layers per block, at least 1024 blocks
  const bool y3d = f.ny > 1;
  const int TX = y3d ? (f.nx < 64 ? f.nx : 64) : (f.nx < 256 ? f.nx : 256);
  const int TY = y3d ? (f.ny < 256 / TX ? f.ny : 256 / TX) : 1;
  const int tiles = (f.nx / TX) * (f.ny / TY);
  int KB = 16;
  while (KB > 2 && ((f.nz + KB - 1) / KB) * tiles < 1024) KB >>= 1;
  if (KB > f.nz) KB = f.nz;
  const int HY = y3d ? TY + 6 : 1;
  // the kernel holds at most 4 (3D) or 2 (2D) tile points and two faces per direction per thread
  const int nth = TX * TY;
  if ((TX + 6) * HY > (y3d ? 4 : 2) * nth || (TX + 1) * TY > 2 * nth || TX * (TY + 1) > 2 * nth)
    return hipErrorInvalidConfiguration;
  const size_t shm = (size_t)((TX + 6) * HY + (TX + 1) * TY + TX * (TY + 1)) * sizeof(T);
  const dim3 grid(f.nx / TX, f.ny / TY, (f.nz + KB - 1) / KB), block(TX, TY, 1);
  if (y3d)
    hipLaunchKernelGGL((k_weno_adv_zm<T, true>), grid, block, shm, st, in.phin, in.phinm1, pv, adv, f.nx,
                       f.ny, f.nz, KB, (T)f.ihx, (T)f.ihy, (T)f.ihz);
  else
    hipLaunchKernelGGL((k_weno_adv_zm<T, false>), grid, block, shm, st, in.phin, in.phinm1, pv, adv, f.nx,
                       f.ny, f.nz, KB, (T)f.ihx, (T)f.ihy, (T)f.ihz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_props_single(const Dims& c, const StepConsts& k, const T* phinew, const T* phin,
                               const T* phinm1, Restricted<T> r, hipStream_t st) {
  const Launch3 L = launch3(c.nx, c.ny, c.nz);
  hipLaunchKernelGGL(k_g_single<T>, L.grid, L.block, 0, st, phinew, phin, phinm1, r, c.nx, c.ny, c.nz,
                     (T)c.ihx, (T)c.ihy, (T)c.ihz, k);
  hipLaunchKernelGGL(k_props_single<T>, L.grid, L.block, 0, st, r, c.nx, c.ny, c.nz, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Dims& f, const Dims& c, const T* u, const T* v, const T* w, T* uf,
                          T* vf, T* wf, hipStream_t st) {
  // first = 1: the star extrapolation reduces to the given level
  Prolonged<T> pv{u, u, v, v, w, w, c.nx, c.ny, c.nz, c.ny == 1 ? 1 : 2, 1, 0};
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
  template hipError_t launch_restrict<T>(const Dims&, const Dims&, const T*, T*, int, hipStream_t); \
  template hipError_t launch_props_single<T>(const Dims&, const StepConsts&, const T*, const T*,   \
                                             const T*, Restricted<T>, hipStream_t);               \
  template hipError_t launch_weno_adv_fine<T>(const Dims&, const Dims&, const StepConsts&, ChIn<T>,  \
                                              T*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
