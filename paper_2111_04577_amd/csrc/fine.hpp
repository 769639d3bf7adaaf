// Fine-grid accessors shared by the phase-field kernels and their adjoint: plain fine views
// and the fine face velocities of eq. dual1 prolonged on the fly from the coarse faces.
#pragma once

#include "kernels.hpp"

namespace drpf {

template <typename T>
struct FineView {
  const T* a;
  int nx, ny, nz;
  __device__ __forceinline__ T at(int k, int j, int i) const {
    return a[(k * ny + wrap(j, ny)) * nx + wrap(i, nx)];
  }
};

// Fine face velocity of the extrapolated coarse field (eq. dual1). Coarse arrays are
// star-extrapolated on the fly: u* = 2 u^n - u^{n-1}, or u^n on the first step.
template <typename T>
struct Prolonged {
  const T *un, *unm1, *vn, *vnm1, *wn, *wnm1;
  int cnx, cny, cnz, ry, first;
  int single;  // 1: single resolution (the phase field on the flow grid: faces as they are)
  __device__ __forceinline__ T star(const T* a, const T* b, int idx) const {
    return first ? a[idx] : (T)2 * a[idx] - b[idx];
  }
  __device__ __forceinline__ int cidx(int k, int j, int i) const {
    return (k * cny + wrap(j, cny)) * cnx + wrap(i, cnx);
  }
  // fine x face I (at x = (I+1) hxf) of fine row (K, J)
  __device__ __forceinline__ T uf(int K, int J, int I) const {
    if (single) return star(un, unm1, cidx(K, J, I));
    const int k = K >> 1, j = ry == 2 ? (J >> 1) : J, i = I >> 1;
    if (I & 1) return star(un, unm1, cidx(k, j, i));
    return (T)0.5 * (star(un, unm1, cidx(k, j, i - 1)) + star(un, unm1, cidx(k, j, i)));
  }
  __device__ __forceinline__ T vf(int K, int J, int I) const {
    if (single) return star(vn, vnm1, cidx(K, J, I));
    const int k = K >> 1, i = I >> 1;
    if (ry == 1) return star(vn, vnm1, cidx(k, 0, i));
    const int j = J >> 1;
    if (J & 1) return star(vn, vnm1, cidx(k, j, i));
    return (T)0.5 * (star(vn, vnm1, cidx(k, j - 1, i)) + star(vn, vnm1, cidx(k, j, i)));
  }
  // fine z face K (at z = (K+1) hzf), K in [-1, 2 cnz - 1]; walls are 0
  __device__ __forceinline__ T wf(int K, int J, int I) const {
    if (single) return (K < 0 || K >= cnz - 1) ? (T)0 : star(wn, wnm1, cidx(K, J, I));
    if (K < 0 || K >= 2 * cnz - 1) return (T)0;
    const int k = K >> 1, j = ry == 2 ? (J >> 1) : J, i = I >> 1;
    if (K & 1) return star(wn, wnm1, cidx(k, j, i));
    const T lo = k > 0 ? star(wn, wnm1, cidx(k - 1, j, i)) : (T)0;
    return (T)0.5 * (lo + star(wn, wnm1, cidx(k, j, i)));
  }
};

}  // namespace drpf
