// Fifth-order WENO-Z face values (Borges, Carmona, Costa, Don 2008, on the third-order
// candidates and smoothness indicators of Jiang and Shu 1996), used by the advection terms of
// eq. NS25 and of the polymer update when the advection scheme is WENO-Z (the scheme the paper
// names for both). Weights alpha_k = d_k (1 + tau5 / (beta_k + eps)), tau5 = |beta_0 - beta_2|,
// d = (1/10, 6/10, 3/10), eps = 1e-40 (1e-30 in FP32, whose arithmetic flushes smaller values).
#pragma once

#include "common.hpp"

namespace drpf {

// a / b: exact in FP64; in FP32 through the hardware reciprocal (within 1 ulp of it), which
// the FP32 form's round-off budget absorbs and which is several times cheaper than IEEE division.
__device__ __forceinline__ double wdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float wdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Value at the face between v0 and vp1, reconstructed from the side of v0.
template <typename T>
__device__ __forceinline__ T weno_face(T vm2, T vm1, T v0, T vp1, T vp2) {
  const T eps = sizeof(T) == 8 ? (T)1e-40 : (T)1e-30;
  const T q0 = ((T)2 * vm2 - (T)7 * vm1 + (T)11 * v0) / (T)6;
  const T q1 = (-vm1 + (T)5 * v0 + (T)2 * vp1) / (T)6;
  const T q2 = ((T)2 * v0 + (T)5 * vp1 - vp2) / (T)6;
  const T c13 = (T)(13.0 / 12.0), c14 = (T)0.25;
  const T s0 = vm2 - (T)2 * vm1 + v0, r0 = vm2 - (T)4 * vm1 + (T)3 * v0;
  const T s1 = vm1 - (T)2 * v0 + vp1, r1 = vm1 - vp1;
  const T s2 = v0 - (T)2 * vp1 + vp2, r2 = (T)3 * v0 - (T)4 * vp1 + vp2;
  const T b0 = c13 * (s0 * s0) + c14 * (r0 * r0);
  const T b1 = c13 * (s1 * s1) + c14 * (r1 * r1);
  const T b2 = c13 * (s2 * s2) + c14 * (r2 * r2);
  const T t5 = fabs(b0 - b2);
  const T a0 = (T)0.1 * ((T)1 + wdiv(t5, b0 + eps));
  const T a1 = (T)0.6 * ((T)1 + wdiv(t5, b1 + eps));
  const T a2 = (T)0.3 * ((T)1 + wdiv(t5, b2 + eps));
  return wdiv(a0 * q0 + a1 * q1 + a2 * q2, a0 + a1 + a2);
}

// Flux u q at the face between cells c0 and p1, with q reconstructed on the upwind side from
// the six cells m2, m1, c0, p1, p2, p3 around the face (a zero velocity carries no flux).
// The stencil is picked by the sign first, so one reconstruction is evaluated, not two.
template <typename T>
__device__ __forceinline__ T weno_flux(T u, T m2, T m1, T c0, T p1, T p2, T p3) {
  const bool pos = u > (T)0;
  return u * weno_face(pos ? m2 : p3, pos ? m1 : p2, pos ? c0 : p1, pos ? p1 : c0, pos ? p2 : m1);
}

// Flux difference F(i+1/2) - F(i-1/2) at cell i from the seven values v[0..6] = cells i-3 ..
// i+3 and the face velocities um (face i-1/2) and up (face i+1/2).
template <typename T>
__device__ __forceinline__ T weno_div1(const T v[7], T um, T up) {
  const T fp = weno_flux(up, v[1], v[2], v[3], v[4], v[5], v[6]);
  const T fm = weno_flux(um, v[0], v[1], v[2], v[3], v[4], v[5]);
  return fp - fm;
}

// Mirror index beyond the walls of an axis of n cells (the homogeneous Neumann extension).
__device__ __forceinline__ int mirror_index(int k, int n) {
  return k < 0 ? -k - 1 : (k >= n ? 2 * n - 1 - k : k);
}

// Byte offsets of the seven cells i-3 .. i+3 along x, y and z (mirrored in z) around cell
// (k, j, i) of a periodic-in-x,y coarse array; shared by every component read with ld_at, so
// each neighbour costs one 32-bit offset rather than a 64-bit address per component.
template <typename T>
struct WenoOffsets {
  unsigned x[7], y[7], z[7];
  __device__ __forceinline__ WenoOffsets(int k, int j, int i, int nx, int ny, int nz) {
#pragma unroll
    for (int d = -3; d <= 3; ++d) {
      x[d + 3] = (unsigned)(((k * ny + j) * nx + wrap(i + d, nx)) * (int)sizeof(T));
      y[d + 3] = (unsigned)(((k * ny + wrap(j + d, ny)) * nx + i) * (int)sizeof(T));
      z[d + 3] = (unsigned)(((mirror_index(k + d, nz) * ny + j) * nx + i) * (int)sizeof(T));
    }
  }
  // -(d(u q)/dx + d(v q)/dy + d(w q)/dz) of the array q at the cell, face velocities given
  __device__ __forceinline__ T advection(const T* q, T um, T up, T vm, T vp, T wm, T wp, T ihx, T ihy,
                                         T ihz) const {
    T vx[7], vy[7], vz[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) {
      vx[d] = ld_at(q, x[d]);
      vy[d] = ld_at(q, y[d]);
      vz[d] = ld_at(q, z[d]);
    }
    return -(weno_div1(vx, um, up) * ihx + weno_div1(vy, vm, vp) * ihy + weno_div1(vz, wm, wp) * ihz);
  }
};

// Byte offsets of the six face neighbours of cell (k, j, i) (x, y periodic; z clamped to the
// domain, the wall terms being zero there), shared by every component read with ld_at.
template <typename T>
struct NbrOffsets {
  unsigned xp, xm, yp, ym, zp, zm;
  __device__ __forceinline__ NbrOffsets(int k, int j, int i, int nx, int ny, int nz) {
    const int es = (int)sizeof(T);
    xp = (unsigned)(((k * ny + j) * nx + wrap(i + 1, nx)) * es);
    xm = (unsigned)(((k * ny + j) * nx + wrap(i - 1, nx)) * es);
    yp = (unsigned)(((k * ny + wrap(j + 1, ny)) * nx + i) * es);
    ym = (unsigned)(((k * ny + wrap(j - 1, ny)) * nx + i) * es);
    zp = (unsigned)((((k < nz - 1 ? k + 1 : k) * ny + j) * nx + i) * es);
    zm = (unsigned)((((k > 0 ? k - 1 : k) * ny + j) * nx + i) * es);
  }
};

}  // namespace drpf
