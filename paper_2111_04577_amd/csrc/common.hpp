// Shared device/host definitions of the drpf HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace drpf {

// ----------------------------------------------------------------------------------------
// complex arithmetic (interleaved re/im, the layout of every spectral buffer)
// ----------------------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) {
  cx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return mk<T>(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return mk<T>(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return mk<T>(s * a.re, s * a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) {
  return mk<T>(a.re, -a.im);
}
// multiply by +i or -i
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  return mk<T>(-a.im, a.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  return mk<T>(a.im, -a.re);
}
template <typename A, typename T>
__host__ __device__ __forceinline__ cx<A> widen(cx<T> a) {
  return mk<A>((A)a.re, (A)a.im);
}

// ----------------------------------------------------------------------------------------
// geometry of one grid (fine or coarse)
// ----------------------------------------------------------------------------------------
struct Dims {
  int nx, ny, nz;       // cells
  int logx, logy;       // log2(nx), log2(ny)
  int pitch;            // nx/2 + 1: complex entries per spectral x-row
  double hx, hy, hz;    // spacings
  double ihx, ihy, ihz; // their reciprocals
  __host__ __device__ size_t cells() const { return (size_t)nx * ny * nz; }
  __host__ __device__ size_t spec() const { return (size_t)pitch * ny * nz; }
  __host__ __device__ int lines() const { return pitch * ny; }
};

// Device tables of one grid: FFT twiddles and spectral eigenvalues.
template <typename T>
struct Tables {
  const cx<T>* tw_xm;    // e^{-2 pi i t / (nx/2)}, t < nx/2 (complex FFT inside r2c/c2r)
  const cx<T>* tw_xn;    // e^{-2 pi i k / nx}, k <= nx/2 (r2c post / c2r pre twiddle)
  const cx<T>* tw_y;     // e^{-2 pi i t / ny}, t < ny
  const double* lam_x;   // -(4/hx^2) sin^2(pi kx / nx), kx <= nx/2
  const double* lam_y;   // -(4/hy^2) sin^2(pi ky / ny), ky < ny
  const double* ph_x;    // (cos, sin)(2 pi kx / nx), kx <= nx/2, interleaved
  const double* ph_y;    // (cos, sin)(2 pi ky / ny), ky < ny, interleaved
  const cx<T>* tw_z;     // e^{-2 pi i t / nz}, t < nz (FFT inside the wall-normal DCT)
  const cx<T>* tw_zq;    // e^{-i pi m / (2 nz)}, m < nz (DCT-II quarter-wave twiddle)
  const double* lam_z;   // -(4/hz^2) sin^2(pi m / (2 nz)), m < nz: DCT-II eigenvalues of the
                         // zero-flux second difference
};

// Scheme constants of one step kind (first step: gamma0 = 1; later: 3/2).
struct StepConsts {
  int first;
  double gamma0, dt;
  double cn, cn2, pe;
  double S, alpha, c_psi;       // Dong splitting (eqs. NS29-NS30)
  double cos_bot, cos_top;      // static contact angles (eq. NS16)
  double rho1, rho2, mu1, mu2;  // drop / ambient density and solvent viscosity
  double rho0, nu_m;            // projection constants (text after eq. NS39)
  double re, k_sigma, c_j;      // 1/Re scaling, capillary coefficient, J = -c_j grad G
  double wi, beta;              // polymer: Weissenberg number, solvent-viscosity ratio
  double ax, ay, az;            // body acceleration
  // reciprocals and products formed once on the host
  double inv_dt, inv_cn2, s_cn2, pe_cn2;  // 1/dt, 1/Cn^2, S/Cn^2, Pe/Cn^2
  double g_bot, g_top;                    // cos(theta) / (sqrt(2) Cn) at each wall
  double inv_re, inv_rho0, inv_wi;
  double giesekus;              // Giesekus mobility alpha (0: Oldroyd-B)
  int advection;                // 0: second-order central flux, 1: WENO-Z (phase field, polymer)
  // wall relaxation (eq. NS34 with D_w > 0): kappa = D_w gamma0 / dt; the wall ghost of phi
  // then carries (kappa / hz)(phi_hat / gamma0 - phi^{n+1}). 0: static contact angle
  double relax_kappa, inv_gamma0;
  // tangential wall velocities (x, y) at z = 0 and z = lz (eq. NS13, u = u_w): the no-slip
  // ghost of u and v is 2 u_w - adjacent
  double uwb[2], uwt[2];
};

// Block shape of the 3D stencil launches: bx threads along x, by along y, one z layer per
// block row of the grid (gridDim.z = nz, or a multiple of it).
struct Launch3 {
  dim3 grid, block;
};
inline Launch3 launch3(int nx, int ny, int nz_blocks, int max_threads = 256) {
  const int bx = nx < 64 ? nx : 64;
  int by = max_threads / bx;
  if (by > ny) by = ny;
  Launch3 l;
  l.block = dim3(bx, by, 1);
  l.grid = dim3(nx / bx, ny / by, nz_blocks);
  return l;
}

// Logical tile of a block under XCD-aware ordering. The hardware hands out blocks
// round-robin over the 8 XCDs of the chip (block b runs on XCD b % 8), and every XCD has
// its own L2. With the grid linearised x-fastest, this sends consecutive tiles -- whose
// halos overlap -- to different L2s. The remap gives XCD x the contiguous logical range
// [x n/8, (x+1) n/8), i.e. its own slab of z layers, so halo re-reads hit its L2.
__device__ __forceinline__ void xcd_tile(int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int nb = gx * gy * gridDim.z;
  const int b = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const int t = (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
  bx = t % gx;
  by = (t / gx) % gy;
  bz = t / (gx * gy);
}

// Layers per block of a z-marching launch over `cols` column tiles: as many blocks as the
// device holds at once (one round, no tail of late blocks), each marching ceil(nz / blocks per
// column) layers.
template <typename K>
inline int march_layers(K kernel, int threads, size_t shm, int cols, int nz) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, shm) != hipSuccess || nb < 1) nb = 1;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    ncu = 1;
  int zb = nb * ncu / cols;
  zb = zb < 1 ? 1 : (zb > nz ? nz : zb);
  return (nz + zb - 1) / zb;
}

// Point q of thread tid in a halo tile of TX x TY interior columns (tid = ty TX + tx) with LO
// halo points before and HI after in x and y, HX = TX + LO + HI wide: point 0 is the thread's
// own interior point, so that a wavefront's first loads cover whole interior rows; points
// 1, 2, ... spread the ring of halo points over the threads (the LO rows below and the HI rows
// above at full width, then the LO columns before and the HI after on each interior row).
// Returns false where the thread has no point q.
template <int LO, int HI>
__device__ __forceinline__ bool own_first_point(int TX, int TY, int tid, int q, int& hy, int& hx) {
  const int HX = TX + LO + HI;
  if (q == 0) {
    hy = tid / TX + LO;
    hx = tid - (hy - LO) * TX + LO;
    return true;
  }
  const int r = tid + (q - 1) * TX * TY;
  const int nrow = (LO + HI) * HX;
  if (r < nrow) {
    const int row = r / HX;
    hx = r - row * HX;
    hy = row < LO ? row : TY + row;
    return true;
  }
  const int s = r - nrow;
  if (s >= (LO + HI) * TY) return false;
  const int c = s % (LO + HI);
  hy = LO + s / (LO + HI);
  hx = c < LO ? c : TX + c;
  return true;
}

// One-dimensional form of xcd_tile: the logical block index, so that consecutive logical
// blocks (which share cache lines) run on the same XCD.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

__host__ __device__ __forceinline__ int wrap(int i, int n) { return i & (n - 1); }

// Element at a byte offset from a base pointer. With a uniform base and a 32-bit per-lane
// offset the load takes the scalar-base + vector-offset form (no 64-bit address per lane).
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_at(T* base, unsigned byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// Streaming stores for the outputs of the z-marching stencils: marked nontemporal, the written
// lines leave L2 first, so more of the halo rows that neighbouring blocks read again stay
// there (at 256 x 256 x 128 coarse cells: 12 % fewer fetched bytes in the polymer RK2 march)
template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}
template <typename T>
__device__ __forceinline__ void st_nt_at(T* base, unsigned byte_off, T v) {
  st_nt(reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off), v);
}

// Spectral layout. After the x transform every z layer holds lines() = (nx/2 + 1) ny modes:
// first the modes kx < nx/2 as ny rows of nx/2 entries (row ky at offset ky nx/2), then the
// Nyquist modes kx = nx/2 of all ky, contiguous. Every array is [z][line]. Rows of a power-of-
// two length keep tiles of consecutive kx (the y transform) on cache-line boundaries, and a
// line's position equals its index, so the wall-normal passes read aligned tiles of
// consecutive lines. Mode (ky, kx) of line l (P = nx/2 + 1):
__device__ __forceinline__ void spec_mode(int l, int P, int Ny, int& ky, int& kx) {
  const int H = P - 1;
  const int main = H * Ny;
  if (l < main) {
    const int lh = __ffs(H) - 1;
    ky = l >> lh;
    kx = l & (H - 1);
  } else {
    kx = H;
    ky = l - main;
  }
}

}  // namespace drpf
