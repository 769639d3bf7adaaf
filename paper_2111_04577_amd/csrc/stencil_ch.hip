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
//                  and edges. A block stages the fine phi^{n+1} tile (with a one-cell halo)
//                  under its coarse tile in LDS, evaluates G once per fine cell of the tile,
//                  then every thread sums its coarse cell's 2x2x2 groups from LDS.
//   prolong, restrict -- the standalone transfer operators (eqs. dual1, dual2).
#include "kernels.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;

template <typename T>
struct FineView {
  const T* a;
  int nx, ny, nz;
  __device__ __forceinline__ T at(int k, int j, int i) const {
    return a[((size_t)k * ny + wrap(j, ny)) * nx + wrap(i, nx)];
  }
};

// Fine face velocity of the extrapolated coarse field (eq. dual1). Coarse arrays are
// star-extrapolated on the fly: u* = 2 u^n - u^{n-1}, or u^n on the first step.
template <typename T>
struct Prolonged {
  const T *un, *unm1, *vn, *vnm1, *wn, *wnm1;
  int cnx, cny, cnz, ry, first;
  __device__ __forceinline__ T star(const T* a, const T* b, size_t idx) const {
    return first ? a[idx] : (T)2 * a[idx] - b[idx];
  }
  __device__ __forceinline__ size_t cidx(int k, int j, int i) const {
    return ((size_t)k * cny + wrap(j, cny)) * cnx + wrap(i, cnx);
  }
  // fine x face I (at x = (I+1) hxf) of fine row (K, J)
  __device__ __forceinline__ T uf(int K, int J, int I) const {
    const int k = K >> 1, j = ry == 2 ? (J >> 1) : J, i = I >> 1;
    if (I & 1) return star(un, unm1, cidx(k, j, i));
    return (T)0.5 * (star(un, unm1, cidx(k, j, i - 1)) + star(un, unm1, cidx(k, j, i)));
  }
  __device__ __forceinline__ T vf(int K, int J, int I) const {
    const int k = K >> 1, i = I >> 1;
    if (ry == 1) return star(vn, vnm1, cidx(k, 0, i));
    const int j = J >> 1;
    if (J & 1) return star(vn, vnm1, cidx(k, j, i));
    return (T)0.5 * (star(vn, vnm1, cidx(k, j - 1, i)) + star(vn, vnm1, cidx(k, j, i)));
  }
  // fine z face K (at z = (K+1) hzf), K in [-1, 2 cnz - 1]; walls are 0
  __device__ __forceinline__ T wf(int K, int J, int I) const {
    if (K < 0 || K >= 2 * cnz - 1) return (T)0;
    const int k = K >> 1, j = ry == 2 ? (J >> 1) : J, i = I >> 1;
    if (K & 1) return star(wn, wnm1, cidx(k, j, i));
    const T lo = k > 0 ? star(wn, wnm1, cidx(k - 1, j, i)) : (T)0;
    return (T)0.5 * (lo + star(wn, wnm1, cidx(k, j, i)));
  }
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_ch_rhs(const T* __restrict__ phin, const T* __restrict__ phinm1, Prolonged<T> pv,
             T* __restrict__ out, int nx, int ny, int nz, T ihx, T ihy, T ihz, StepConsts c) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int I = bx * blockDim.x + threadIdx.x;
  const int J = by * blockDim.y + threadIdx.y;
  const int K = bz;
  const FineView<T> A{phin, nx, ny, nz}, B{phinm1, nx, ny, nz};
  const bool first = c.first != 0;
  auto star = [&](int k, int j, int i) -> T {
    return first ? A.at(k, j, i) : (T)2 * A.at(k, j, i) - B.at(k, j, i);
  };
  const T ihx2 = ihx * ihx, ihy2 = ihy * ihy, ihz2 = ihz * ihz;
  // phi* on the 7-point stencil, zero-flux ghosts in z
  const T p0 = star(K, J, I);
  const T pxp = star(K, J, I + 1), pxm = star(K, J, I - 1);
  const T pyp = star(K, J + 1, I), pym = star(K, J - 1, I);
  const T pzp = K + 1 < nz ? star(K + 1, J, I) : p0;
  const T pzm = K > 0 ? star(K - 1, J, I) : p0;
  const T phat = first ? A.at(K, J, I) : (T)2 * A.at(K, J, I) - (T)0.5 * B.at(K, J, I);
  // advection div(u_f* phi*) in flux form, zero wall flux
  const T h = (T)0.5;
  const T fxp = pv.uf(K, J, I) * h * (p0 + pxp);
  const T fxm = pv.uf(K, J, I - 1) * h * (pxm + p0);
  const T fyp = pv.vf(K, J, I) * h * (p0 + pyp);
  const T fym = pv.vf(K, J - 1, I) * h * (pym + p0);
  const T fzp = K + 1 < nz ? pv.wf(K, J, I) * h * (p0 + pzp) : (T)0;
  const T fzm = K > 0 ? pv.wf(K - 1, J, I) * h * (pzm + p0) : (T)0;
  const T adv = (fxp - fxm) * ihx + (fyp - fym) * ihy + (fzp - fzm) * ihz;
  // w* = f(phi*) - (S/Cn^2) phi*,   f = (phi^3 - phi) / Cn^2
  const T icn2 = (T)c.inv_cn2, sc = (T)c.s_cn2;
  auto wst = [&](T p) -> T { return (p * p * p - p) * icn2 - sc * p; };
  const T w0 = wst(p0);
  const T lapw = (wst(pxp) - 2 * w0 + wst(pxm)) * ihx2 + (wst(pyp) - 2 * w0 + wst(pym)) * ihy2 +
                 (wst(pzp) - 2 * w0 + wst(pzm)) * ihz2;
  // wetting data b = g(phi*_wall) / hz on the wall-adjacent layers, and L_N b
  const T gb = (T)c.g_bot * ihz, gt = (T)c.g_top * ihz;
  auto bval = [&](int k, T p) -> T {
    T b = 0;
    if (k == 0) b += gb * ((T)1 - p * p);
    if (k == nz - 1) b += gt * ((T)1 - p * p);
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
    // an interior layer next to a wall layer sees b of that layer through its z neighbour
    if (K == 1) lapb += bval(0, pzm) * ihz2;
    if (K == nz - 2) lapb += bval(nz - 1, pzp) * ihz2;
  }
  const T q = (T)c.pe_cn2 * (phat * (T)c.inv_dt - adv) + lapw;
  out[((size_t)K * ny + J) * nx + I] = q - lapb;
}

// Per-axis weights of the 1D restriction rules for a fine offset d relative to r * i
// (r the refinement factor of that axis): centre rule and face rule.
__device__ __forceinline__ float wc(int d, int r) { return r == 2 ? (d < 2 ? 0.5f : 0.f) : (d == 0 ? 1.f : 0.f); }
__device__ __forceinline__ float wf(int d, int r) { return r == 2 ? (d >= 1 ? 0.5f : 0.f) : (d <= 1 ? 0.5f : 0.f); }

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_restrict_g(const T* __restrict__ phinew, const T* __restrict__ phin,
                 const T* __restrict__ phinm1, Restricted<T> r, int fnx, int fny, int fnz,
                 T fihx, T fihy, T fihz, int cnx, int cny, int cnz, int ry, int KZ,
                 StepConsts c) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int CX = blockDim.x, CY = blockDim.y;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i0 = bx * CX, j0 = by * CY, k0 = bz * KZ;
  // G region: fine x 2 i0 .. 2 i0 + 2 CX, y ry j0 .. ry j0 + ry CY, z 2 k0 .. 2 k0 + 2 KZ
  // (clamped to the top layer); phi^{n+1} tile one cell wider on every side.
  const int GX = 2 * CX + 1, GY = ry * CY + 1, GZ = 2 * KZ + 1;
  const int PX = GX + 2, PY = GY + 2, PZ = GZ + 2;
  const int X0 = 2 * i0, Y0 = ry * j0, Z0 = 2 * k0;
  T* sP = reinterpret_cast<T*>(smem);  // phi^{n+1} on the halo tile, layers clamp(Z0 - 1 + pz)
  T* sG = sP + PX * PY * PZ;           // G on the G region
  const int tid = threadIdx.y * CX + threadIdx.x;
  const int nth = CX * CY;
  const FineView<T> N{phinew, fnx, fny, fnz}, A{phin, fnx, fny, fnz}, B{phinm1, fnx, fny, fnz};
  for (int e = tid; e < PX * PY * PZ; e += nth) {
    const int pz = e / (PX * PY);
    const int rem = e - pz * PX * PY;
    const int py = rem / PX;
    const int px = rem - py * PX;
    const int Kz = min(max(Z0 - 1 + pz, 0), fnz - 1);
    sP[e] = N.at(Kz, Y0 - 1 + py, X0 - 1 + px);
  }
  __syncthreads();
  const bool first = c.first != 0;
  const T ihx2 = fihx * fihx, ihy2 = fihy * fihy, ihz2 = fihz * fihz;
  const T cn2 = (T)c.cn2, S = (T)c.S;
  const T gb = (T)c.g_bot * fihz, gt = (T)c.g_top * fihz;
  auto pzi = [&](int Kf) { return min(max(Kf, 0), fnz - 1) - Z0 + 1; };
  auto P = [&](int pz, int py, int px) -> T { return sP[(pz * PY + py) * PX + px]; };
  for (int e = tid; e < GX * GY * GZ; e += nth) {
    const int gz = e / (GX * GY);
    const int rem = e - gz * GX * GY;
    const int gy = rem / GX;
    const int gx = rem - gy * GX;
    const int K = min(Z0 + gz, fnz - 1);
    const int pz = pzi(K), py = gy + 1, px = gx + 1;
    const T p = P(pz, py, px);
    const T lap = (P(pz, py, px + 1) - 2 * p + P(pz, py, px - 1)) * ihx2 +
                  (P(pz, py + 1, px) - 2 * p + P(pz, py - 1, px)) * ihy2 +
                  (P(pzi(K + 1), py, px) - 2 * p + P(pzi(K - 1), py, px)) * ihz2;
    const T an = A.at(K, Y0 + gy, X0 + gx);
    const T ps = first ? an : (T)2 * an - B.at(K, Y0 + gy, X0 + gx);
    T b = 0;
    if (K == 0) b += gb * ((T)1 - ps * ps);
    if (K == fnz - 1) b += gt * ((T)1 - ps * ps);
    sG[e] = -cn2 * (lap + b) + S * (p - ps) + ps * ps * ps - ps;
  }
  __syncthreads();
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = i0 + tx, j = j0 + ty;
  for (int kk = 0; kk < KZ; ++kk) {
  const int k = k0 + kk;
  T phic = 0, Gc = 0, phx = 0, Gx = 0, phy = 0, Gy = 0, phz = 0, Gz = 0;
  T phxy = 0, phxz = 0, phyz = 0, phxz_b = 0, phyz_b = 0;
  const int ndy = ry + 1;
  for (int dz = 0; dz < 3; ++dz) {
    const int gz = 2 * kk + dz;
    const int K = min(Z0 + gz, fnz - 1);
    const int pz = pzi(K);
    const T zc = (T)wc(dz, 2), zf = (T)wf(dz, 2);
    for (int dy = 0; dy < ndy; ++dy) {
      const int gy = ry * ty + dy;
      const T yc = (T)wc(dy, ry), yf = (T)wf(dy, ry);
      for (int dx = 0; dx < 3; ++dx) {
        const int gx = 2 * tx + dx;
        const T p = P(pz, gy + 1, gx + 1);
        const T G = sG[(gz * GY + gy) * GX + gx];
        const T xc = (T)wc(dx, 2), xf = (T)wf(dx, 2);
        phic += xc * yc * zc * p;
        Gc += xc * yc * zc * G;
        phx += xf * yc * zc * p;
        Gx += xf * yc * zc * G;
        phy += xc * yf * zc * p;
        Gy += xc * yf * zc * G;
        phz += xc * yc * zf * p;
        Gz += xc * yc * zf * G;
        phxy += xf * yf * zc * p;
        phxz += xf * yc * zf * p;
        phyz += xc * yf * zf * p;
        if (dz == 0) {
          phxz_b += xf * yc * p;
          phyz_b += xc * yf * p;
        }
      }
    }
  }
  const T r1 = (T)c.rho1, r2 = (T)c.rho2, m1 = (T)c.mu1, m2 = (T)c.mu2, hf = (T)0.5;
  auto rinv = [&](T ph) { return (T)1 / (hf * ((T)1 + ph) * r1 + hf * ((T)1 - ph) * r2); };
  auto mu = [&](T ph) { return hf * ((T)1 + ph) * m1 + hf * ((T)1 - ph) * m2; };
  const size_t id = ((size_t)k * cny + j) * cnx + i;
  r.phi_c[id] = phic;
  r.G_c[id] = Gc;
  r.G_x[id] = Gx;
  r.G_y[id] = Gy;
  r.G_z[id] = Gz;
  r.ri_x[id] = rinv(phx);
  r.ri_y[id] = rinv(phy);
  r.ri_z[id] = rinv(phz);
  r.mu_c[id] = mu(phic);
  r.mu_xy[id] = mu(phxy);
  // z-edge arrays carry nz + 1 layers: layer k + 1 is the edge at z = (k + 1) hz
  const size_t plane = (size_t)cnx * cny;
  r.mu_xz[id + plane] = mu(phxz);
  r.mu_yz[id + plane] = mu(phyz);
  if (k == 0) {
    r.mu_xz[id] = mu(phxz_b);
    r.mu_yz[id] = mu(phyz_b);
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
  const Launch3 L = launch3(f.nx, f.ny, f.nz);
  hipLaunchKernelGGL(k_ch_rhs<T>, L.grid, L.block, 0, st, in.phin, in.phinm1, pv, rhs, f.nx, f.ny,
                     f.nz, (T)f.ihx, (T)f.ihy, (T)f.ihz, k);
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
  // coarse layers per block (the kernel supports KZ > 1, which amortises the z halo, but on
  // gfx950 the larger LDS tile lowers occupancy more than it saves: one layer measures best)
  const int KZ = 1;
  const int GX = 2 * CX + 1, GY = ry * CY + 1, GZ = 2 * KZ + 1;
  const size_t shm = (size_t)((GX + 2) * (GY + 2) * (GZ + 2) + GX * GY * GZ) * sizeof(T);
  hipLaunchKernelGGL(k_restrict_g<T>, dim3(c.nx / CX, c.ny / CY, c.nz / KZ), dim3(CX, CY, 1), shm, st,
                     phinew, phin, phinm1, r, f.nx, f.ny, f.nz, (T)f.ihx, (T)f.ihy, (T)f.ihz, c.nx,
                     c.ny, c.nz, ry, KZ, k);
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
