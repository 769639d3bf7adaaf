// FP64 observables of a state: phase-field mass (the conserved quantity of Sec. 3.2.1),
// wetted radius and centroid height of the drop phase, kinetic energy and max |div u|.
// Deterministic: fixed-size grid, fixed per-thread strides, fixed-order block tree, one
// finishing block; no floating-point atomics, so repeated calls give identical bits.
#include "kernels.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;
constexpr int kBlocks = 512;
constexpr int kQ = 6;  // fine sums: phi, ind, z*ind, wall ind, nonfinite; coarse: ke (max div separate)

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_obs_partial(const T* __restrict__ phi, int fnx, int fny, int fnz, double fhz,
                  const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w, int cnx,
                  int cny, int cnz, double hx, double hy, double hz, double* __restrict__ part) {
  __shared__ double sh[kBlock];
  const size_t nf = (size_t)fnx * fny * fnz;
  const size_t plane = (size_t)fnx * fny;
  const size_t stride = (size_t)kBlocks * kBlock;
  double s_phi = 0, s_ind = 0, s_zind = 0, s_wall = 0, bad = 0;
  for (size_t id = (size_t)blockIdx.x * kBlock + threadIdx.x; id < nf; id += stride) {
    const double p = (double)phi[id];
    if (!isfinite(p)) bad += 1.0;
    const double ind = 0.5 * (1.0 + p);
    const int K = (int)(id / plane);
    s_phi += p;
    s_ind += ind;
    s_zind += ((double)K + 0.5) * fhz * ind;
    if (K == 0) s_wall += ind;
  }
  const size_t nc = (size_t)cnx * cny * cnz;
  double s_ke = 0, m_div = 0;
  for (size_t id = (size_t)blockIdx.x * kBlock + threadIdx.x; id < nc; id += stride) {
    const int i = (int)(id % cnx);
    const int j = (int)((id / cnx) % cny);
    const int k = (int)(id / ((size_t)cnx * cny));
    const double uu = (double)u[id], vv = (double)v[id], ww = (double)w[id];
    s_ke += uu * uu + vv * vv + ww * ww;
    const double um = (double)u[((size_t)k * cny + j) * cnx + wrap(i - 1, cnx)];
    const double vm = (double)v[((size_t)k * cny + wrap(j - 1, cny)) * cnx + i];
    const double wm = k > 0 ? (double)w[id - (size_t)cnx * cny] : 0.0;
    const double d = (uu - um) / hx + (vv - vm) / hy + (ww - wm) / hz;
    m_div = fmax(m_div, fabs(d));
  }
  double vals[kQ] = {s_phi, s_ind, s_zind, s_wall, bad, s_ke};
  for (int q = 0; q < kQ; ++q) {
    const double r = block_sum(vals[q], sh);
    if (threadIdx.x == 0) part[q * kBlocks + blockIdx.x] = r;
  }
  const double r = block_max(m_div, sh);
  if (threadIdx.x == 0) part[kQ * kBlocks + blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock)
    k_obs_final(const double* __restrict__ part, double* __restrict__ out, double fhx, double fhy,
                double fhz, double chx, double chy, double chz, int two_d) {
  __shared__ double sh[kBlock];
  double tot[kQ + 1];
  for (int q = 0; q < kQ; ++q) {
    double s = 0;
    for (int b = threadIdx.x; b < kBlocks; b += kBlock) s += part[q * kBlocks + b];
    tot[q] = block_sum(s, sh);
  }
  double m = 0;
  for (int b = threadIdx.x; b < kBlocks; b += kBlock) m = fmax(m, part[kQ * kBlocks + b]);
  tot[kQ] = block_max(m, sh);
  if (threadIdx.x == 0) {
    out[0] = tot[0] * fhx * fhy * fhz;
    out[1] = two_d ? 0.5 * fhx * tot[3] : sqrt(fhx * fhy * tot[3] / 3.14159265358979323846);
    out[2] = tot[2] / tot[1];
    out[3] = 0.5 * tot[5] * chx * chy * chz;
    out[4] = tot[kQ];
    out[5] = tot[4];  // count of non-finite phase-field values
  }
}

}  // namespace

size_t reduce_partials() { return (size_t)(kQ + 1) * kBlocks; }

template <typename T>
hipError_t launch_observables(const Dims& f, const Dims& c, const T* phi, const T* u, const T* v,
                              const T* w, double* partial, double* out_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_obs_partial<T>, dim3(kBlocks), dim3(kBlock), 0, st, phi, f.nx, f.ny, f.nz,
                     f.hz, u, v, w, c.nx, c.ny, c.nz, c.hx, c.hy, c.hz, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(kBlock), 0, st, partial, out_dev, f.hx, f.hy, f.hz,
                     c.hx, c.hy, c.hz, c.ny == 1 ? 1 : 0);
  return hipGetLastError();
}

#define INST(T)                                                                                 \
  template hipError_t launch_observables<T>(const Dims&, const Dims&, const T*, const T*,       \
                                            const T*, const T*, double*, double*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
