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
//                  and edges.
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
    const int k = K >> 1, j = J / ry, i = I >> 1;
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
    const int k = K >> 1, j = J / ry, i = I >> 1;
    if (K & 1) return star(wn, wnm1, cidx(k, j, i));
    const T lo = k > 0 ? star(wn, wnm1, cidx(k - 1, j, i)) : (T)0;
    return (T)0.5 * (lo + star(wn, wnm1, cidx(k, j, i)));
  }
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_ch_rhs(const T* __restrict__ phin, const T* __restrict__ phinm1, Prolonged<T> pv,
             T* __restrict__ out, int nx, int ny, int nz, double hx, double hy, double hz,
             StepConsts c) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)nx * ny * nz;
  if (id >= n) return;
  const int I = (int)(id % nx);
  const int J = (int)((id / nx) % ny);
  const int K = (int)(id / ((size_t)nx * ny));
  const FineView<T> A{phin, nx, ny, nz}, B{phinm1, nx, ny, nz};
  const bool first = c.first != 0;
  auto star = [&](int k, int j, int i) -> T {
    return first ? A.at(k, j, i) : (T)2 * A.at(k, j, i) - B.at(k, j, i);
  };
  const T ihx2 = (T)(1.0 / (hx * hx)), ihy2 = (T)(1.0 / (hy * hy)), ihz2 = (T)(1.0 / (hz * hz));
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
  const T adv = (fxp - fxm) * (T)(1.0 / hx) + (fyp - fym) * (T)(1.0 / hy) + (fzp - fzm) * (T)(1.0 / hz);
  // w* = f(phi*) - (S/Cn^2) phi*,   f = (phi^3 - phi) / Cn^2
  const T icn2 = (T)(1.0 / c.cn2), sc = (T)(c.S / c.cn2);
  auto wst = [&](T p) -> T { return (p * p * p - p) * icn2 - sc * p; };
  const T w0 = wst(p0);
  const T lapw = (wst(pxp) - 2 * w0 + wst(pxm)) * ihx2 + (wst(pyp) - 2 * w0 + wst(pym)) * ihy2 +
                 (wst(pzp) - 2 * w0 + wst(pzm)) * ihz2;
  // wetting data b = g(phi*_wall) / hz on the wall-adjacent layers; L_N b
  const T sq2cn = (T)(1.0 / (1.41421356237309504880 * c.cn));
  const T ihz = (T)(1.0 / hz);
  auto bval = [&](int k, T p) -> T {
    T b = 0;
    if (k == 0) b += (T)c.cos_bot * ((T)1 - p * p) * sq2cn * ihz;
    if (k == nz - 1) b += (T)c.cos_top * ((T)1 - p * p) * sq2cn * ihz;
    return b;
  };
  T lapb = 0;
  if (K == 0 || K == nz - 1) {
    const T b0 = bval(K, p0);
    lapb += (bval(K, pxp) - 2 * b0 + bval(K, pxm)) * ihx2 + (bval(K, pyp) - 2 * b0 + bval(K, pym)) * ihy2;
    // z part: neighbours inside the domain carry b only if they are wall layers too
    const T bup = K + 1 < nz ? bval(K + 1, pzp) : b0;
    const T bdn = K > 0 ? bval(K - 1, pzm) : b0;
    lapb += (bup - 2 * b0 + bdn) * ihz2;
  }
  if (K == 1 || K == nz - 2) {
    // z neighbour on a wall layer contributes b there
    T bz = 0;
    if (K == 1) bz += bval(0, pzm);
    if (K == nz - 2) bz += bval(nz - 1, pzp);
    if (!(K == 0 || K == nz - 1)) lapb += bz * ihz2;
  }
  const T q = (T)(c.pe / c.cn2) * (phat * (T)(1.0 / c.dt) - adv) + lapw;
  out[id] = q - lapb;
}

// Per-axis weights of the 1D restriction rules for a fine offset d in {0, 1, 2} relative
// to r * i (r the refinement factor of that axis).
__device__ __forceinline__ double wc(int d, int r) { return r == 2 ? (d < 2 ? 0.5 : 0.0) : (d == 0 ? 1.0 : 0.0); }
__device__ __forceinline__ double wf(int d, int r) { return r == 2 ? (d >= 1 ? 0.5 : 0.0) : (d <= 1 ? 0.5 : 0.0); }

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_restrict_g(const T* __restrict__ phinew, const T* __restrict__ phin,
                 const T* __restrict__ phinm1, Restricted<T> r, int fnx, int fny, int fnz,
                 double hx, double hy, double hz, int cnx, int cny, int cnz, int ry, StepConsts c) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nc = (size_t)cnx * cny * cnz;
  if (id >= nc) return;
  const int i = (int)(id % cnx);
  const int j = (int)((id / cnx) % cny);
  const int k = (int)(id / ((size_t)cnx * cny));
  const FineView<T> N{phinew, fnx, fny, fnz}, A{phin, fnx, fny, fnz}, B{phinm1, fnx, fny, fnz};
  const bool first = c.first != 0;
  const double ihx2 = 1.0 / (hx * hx), ihy2 = 1.0 / (hy * hy), ihz2 = 1.0 / (hz * hz);
  const double sq2cn = 1.0 / (1.41421356237309504880 * c.cn);
  double phic = 0, Gc = 0, phx = 0, Gx = 0, phy = 0, Gy = 0, phz = 0, Gz = 0;
  double phxy = 0, phxz = 0, phyz = 0, phxz_b = 0, phyz_b = 0;
  const int ny_off = ry == 2 ? 3 : 2;
  for (int dz = 0; dz < 3; ++dz) {
    const int K = min(2 * k + dz, fnz - 1);
    for (int dy = 0; dy < ny_off; ++dy) {
      const int J = ry * j + dy;
      for (int dx = 0; dx < 3; ++dx) {
        const int I = 2 * i + dx;
        const double p = (double)N.at(K, J, I);
        const double pxp = N.at(K, J, I + 1), pxm = N.at(K, J, I - 1);
        const double pyp = N.at(K, J + 1, I), pym = N.at(K, J - 1, I);
        const double pzp = K + 1 < fnz ? (double)N.at(K + 1, J, I) : p;
        const double pzm = K > 0 ? (double)N.at(K - 1, J, I) : p;
        const double lap = (pxp - 2 * p + pxm) * ihx2 + (pyp - 2 * p + pym) * ihy2 + (pzp - 2 * p + pzm) * ihz2;
        const double ps = first ? (double)A.at(K, J, I) : 2.0 * (double)A.at(K, J, I) - (double)B.at(K, J, I);
        double b = 0;
        if (K == 0) b += c.cos_bot * (1.0 - ps * ps) * sq2cn / hz;
        if (K == fnz - 1) b += c.cos_top * (1.0 - ps * ps) * sq2cn / hz;
        const double G = -c.cn2 * (lap + b) + c.S * (p - ps) + ps * ps * ps - ps;
        const double xc = wc(dx, 2), xf = wf(dx, 2);
        const double yc = wc(dy, ry), yf = wf(dy, ry);
        const double zc = wc(dz, 2), zf = wf(dz, 2);
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
  auto rho = [&](double ph) { return 0.5 * (1.0 + ph) * c.rho1 + 0.5 * (1.0 - ph) * c.rho2; };
  auto mu = [&](double ph) { return 0.5 * (1.0 + ph) * c.mu1 + 0.5 * (1.0 - ph) * c.mu2; };
  r.phi_c[id] = (T)phic;
  r.G_c[id] = (T)Gc;
  r.G_x[id] = (T)Gx;
  r.G_y[id] = (T)Gy;
  r.G_z[id] = (T)Gz;
  r.ri_x[id] = (T)(1.0 / rho(phx));
  r.ri_y[id] = (T)(1.0 / rho(phy));
  r.ri_z[id] = (T)(1.0 / rho(phz));
  r.mu_c[id] = (T)mu(phic);
  r.mu_xy[id] = (T)mu(phxy);
  // z-edge arrays carry nz + 1 layers: layer k + 1 is the edge at z = (k + 1) hz
  const size_t plane = (size_t)cnx * cny;
  r.mu_xz[id + plane] = (T)mu(phxz);
  r.mu_yz[id + plane] = (T)mu(phyz);
  if (k == 0) {
    r.mu_xz[id] = (T)mu(phxz_b);
    r.mu_yz[id] = (T)mu(phyz_b);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_prolong(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
              T* __restrict__ uf, T* __restrict__ vf, T* __restrict__ wf, int fnx, int fny, int fnz,
              Prolonged<T> pv) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)fnx * fny * fnz;
  if (id >= n) return;
  const int I = (int)(id % fnx);
  const int J = (int)((id / fnx) % fny);
  const int K = (int)(id / ((size_t)fnx * fny));
  uf[id] = pv.uf(K, J, I);
  vf[id] = pv.vf(K, J, I);
  wf[id] = pv.wf(K, J, I);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_restrict(const T* __restrict__ f, T* __restrict__ out, int fnx, int fny, int fnz, int cnx,
               int cny, int cnz_out, int ry, int lx, int ly, int lz) {
  // lx/ly/lz: 0 centre-located, 1 face-located along that axis. A face-located z output has
  // cnz + 1 layers; layer m is the face at z = m hz (m = 0 the bottom wall).
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)cnx * cny * cnz_out;
  if (id >= n) return;
  const int i = (int)(id % cnx);
  const int j = (int)((id / cnx) % cny);
  const int m = (int)(id / ((size_t)cnx * cny));
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
  out[id] = (T)s;
}

}  // namespace

template <typename T>
hipError_t launch_ch_rhs(const Dims& f, const Dims& c, const StepConsts& k, ChIn<T> in, T* rhs,
                         hipStream_t st) {
  Prolonged<T> pv{in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1, c.nx, c.ny, c.nz,
                  c.ny == 1 ? 1 : 2, k.first};
  const size_t n = f.cells();
  hipLaunchKernelGGL(k_ch_rhs<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     in.phin, in.phinm1, pv, rhs, f.nx, f.ny, f.nz, f.hx, f.hy, f.hz, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_g(const Dims& f, const Dims& c, const StepConsts& k, const T* phinew,
                             const T* phin, const T* phinm1, Restricted<T> r, hipStream_t st) {
  const size_t n = c.cells();
  hipLaunchKernelGGL(k_restrict_g<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     st, phinew, phin, phinm1, r, f.nx, f.ny, f.nz, f.hx, f.hy, f.hz, c.nx, c.ny,
                     c.nz, c.ny == 1 ? 1 : 2, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Dims& f, const Dims& c, const T* u, const T* v, const T* w, T* uf,
                          T* vf, T* wf, hipStream_t st) {
  // first = 1: the star extrapolation reduces to the given level
  Prolonged<T> pv{u, u, v, v, w, w, c.nx, c.ny, c.nz, c.ny == 1 ? 1 : 2, 1};
  const size_t n = f.cells();
  hipLaunchKernelGGL(k_prolong<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     u, v, w, uf, vf, wf, f.nx, f.ny, f.nz, pv);
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
  const size_t n = (size_t)c.nx * c.ny * nzo;
  hipLaunchKernelGGL(k_restrict<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     fine, coarse, f.nx, f.ny, f.nz, c.nx, c.ny, nzo, c.ny == 1 ? 1 : 2, lx, ly, lz);
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
