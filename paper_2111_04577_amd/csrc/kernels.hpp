// Host-side launchers of the drpf kernels. Every launcher queues work on `st` and
// returns hipSuccess or the launch error.
#pragma once

#include "common.hpp"

namespace drpf {

// Up to four fields processed by one transform launch (fields are consecutive batches of
// nz*ny lines). For the inverse x transform, add[f] (if not null) is added to the output.
template <typename T>
struct RealSet {
  T* p[4];
  const T* add[4];
  int nfields;
};

// ---- fft.hip --------------------------------------------------------------------------
template <typename T>
hipError_t launch_fft_x_fwd(const Dims& d, const Tables<T>& tb, const T* const in[4], int nfields,
                            cx<T>* spec, hipStream_t st);
template <typename T>
hipError_t launch_fft_x_inv(const Dims& d, const Tables<T>& tb, const cx<T>* spec, RealSet<T> out,
                            hipStream_t st);
template <typename T>
hipError_t launch_fft_y(const Dims& d, const Tables<T>& tb, cx<T>* spec, int nfields, bool inverse,
                        hipStream_t st);

// ---- tridiag.hip ----------------------------------------------------------------------
// bc: 0 Neumann, 1 Dirichlet (centred), 2 Dirichlet (z faces). Solves coeff L x - shift x =
// (scale * spec) in place per Fourier mode; Neumann with shift 0 pins the zero mode and
// removes its mean.
template <typename T>
hipError_t launch_zpass_helmholtz(const Dims& d, const Tables<T>& tb, cx<T>* spec, double* piv,
                                  int bc, double coeff, double shift, double scale, hipStream_t st);
// Cahn-Hilliard: (L - c_psi) then (L + alpha), both Neumann.
template <typename T>
hipError_t launch_zpass_ch(const Dims& d, const Tables<T>& tb, cx<T>* spec, double* piv,
                           double c_psi, double alpha, double scale, hipStream_t st);
// Navier-Stokes: velocity Helmholtz x3, divergence, FP64 Poisson, correction.
template <typename T>
hipError_t launch_zpass_ns(const Dims& d, const Tables<T>& tb, cx<T>* spec4, double* piv,
                           const StepConsts& c, double scale, hipStream_t st);

// ---- stencil_ch.hip -------------------------------------------------------------------
template <typename T>
struct ChIn {
  const T* phin;
  const T* phinm1;
  const T *un, *unm1, *vn, *vnm1, *wn, *wnm1;  // coarse faces
};
template <typename T>
hipError_t launch_ch_rhs(const Dims& f, const Dims& c, const StepConsts& k, ChIn<T> in, T* rhs,
                         hipStream_t st);

// Restricted coarse set written by launch_restrict_g.
template <typename T>
struct Restricted {
  T *phi_c, *G_c, *G_x, *G_y, *G_z, *ri_x, *ri_y, *ri_z, *mu_c, *mu_xy, *mu_xz, *mu_yz;
};
template <typename T>
hipError_t launch_restrict_g(const Dims& f, const Dims& c, const StepConsts& k, const T* phinew,
                             const T* phin, const T* phinm1, Restricted<T> r, hipStream_t st);
template <typename T>
hipError_t launch_prolong(const Dims& f, const Dims& c, const T* u, const T* v, const T* w, T* uf,
                          T* vf, T* wf, hipStream_t st);
template <typename T>
hipError_t launch_restrict(const Dims& f, const Dims& c, const T* fine, T* coarse, int location,
                           hipStream_t st);

// ---- stencil_ns.hip -------------------------------------------------------------------
template <typename T>
struct NsIn {
  const T *un, *unm1, *vn, *vnm1, *wn, *wnm1, *pn, *pnm1;
  const T* taun[6];
  const T* taunm1[6];
  int viscoelastic;
};
template <typename T>
hipError_t launch_momentum_rhs(const Dims& c, const StepConsts& k, NsIn<T> in, Restricted<T> r,
                               T* ru, T* rv, T* rw, hipStream_t st);
// One RK2-TVD stage: out = c0 * tau_n + c1 * (tau_in + dt RH(tau_in)), u fixed.
template <typename T>
hipError_t launch_polymer_stage(const Dims& c, const StepConsts& k, const T* u, const T* v,
                                const T* w, const T* const tau_n[6], const T* const tau_in[6],
                                T* const tau_out[6], double c0, double c1, hipStream_t st);

// ---- reduce.hip -----------------------------------------------------------------------
// Writes DRPF_OBS_COUNT doubles to out_dev (device), using `partial` (device scratch of
// reduce_partials() doubles). Returns also a non-finite flag in out_dev[DRPF_OBS_COUNT].
template <typename T>
hipError_t launch_observables(const Dims& f, const Dims& c, const T* phi, const T* u, const T* v,
                              const T* w, double* partial, double* out_dev, hipStream_t st);
size_t reduce_partials();

}  // namespace drpf
