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
// The x and y passes in one kernel, a block per layer of a field (coarse layers that fit in
// a block's LDS; fft_xy_fits says whether they do).
template <typename T>
bool fft_xy_fits(const Dims& d);
template <typename T>
hipError_t launch_fft_xy_fwd(const Dims& d, const Tables<T>& tb, const T* const in[4], int nfields,
                             cx<T>* spec, hipStream_t st);
template <typename T>
hipError_t launch_fft_xy_inv(const Dims& d, const Tables<T>& tb, const cx<T>* spec, RealSet<T> out,
                             hipStream_t st);

// ---- tridiag.hip ----------------------------------------------------------------------
// bc: 0 Neumann, 1 Dirichlet (centred), 2 Dirichlet (z faces). Solves coeff L x - shift x =
// (scale * spec) in place per Fourier mode; Neumann with shift 0 pins the zero mode and
// removes its mean.
template <typename T>
hipError_t launch_zpass_helmholtz(const Dims& d, const Tables<T>& tb, cx<T>* spec, int bc,
                                  double coeff, double shift, double scale, hipStream_t st);
// Wall data of a solve moved to its right-hand side: out = rhs - coeff b, b nonzero on the
// layers next to the walls (bc 0: wall[] = outward normal derivative g, b = g / hz; bc 1: wall
// value, b = 2 wall / hz^2; bc 2: wall value of the face field, b = wall / hz^2 on faces 0 and
// nz-2, and layer nz-1 of out is 0). wall holds the bottom then the top x-y layer.
template <typename T>
hipError_t launch_wall_rhs(const Dims& d, int bc, double coeff, const T* rhs, const T* wall, T* out,
                           hipStream_t st);
// x[nz-1][.][.] = top (one x-y layer)
template <typename T>
hipError_t launch_top_layer(const Dims& d, const T* top, T* x, hipStream_t st);
// Cahn-Hilliard: (L - c_psi) then (L + alpha), both Neumann; with dwall != 0 the fused
// operator gains L dW (dW: dwall on the two wall-adjacent rows), the relaxed walls of eq. NS34.
// trans (FP64, dwall != 0): the transposed operator, (L - c_psi)(L + alpha) + dW L.
template <typename T>
hipError_t launch_zpass_ch(const Dims& d, const Tables<T>& tb, cx<T>* spec, double c_psi,
                           double alpha, double scale, double dwall, hipStream_t st, bool trans = false);
// Navier-Stokes: velocity Helmholtz x3, divergence, FP64 Poisson, correction.
template <typename T>
hipError_t launch_zpass_ns(const Dims& d, const Tables<T>& tb, cx<T>* spec4, const StepConsts& c,
                           double scale, hipStream_t st);

// ---- stencil_ch.hip -------------------------------------------------------------------
template <typename T>
struct ChIn {
  const T* phin;
  const T* phinm1;
  const T *un, *unm1, *vn, *vnm1, *wn, *wnm1;  // coarse faces
  const T* adv;  // if not null: div(u phi*) precomputed (WENO-Z), fine cells
};
// div(u_f phi*) on the fine grid with WENO-Z face values (the advection of eq. NS25 in the
// paper's scheme), into adv (fine cells).
template <typename T>
hipError_t launch_weno_adv_fine(const Dims& f, const Dims& c, const StepConsts& k, ChIn<T> in, T* adv,
                                hipStream_t st);
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
// Single resolution: the restricted set from the phase field on the flow grid (c = the grid).
template <typename T>
hipError_t launch_props_single(const Dims& c, const StepConsts& k, const T* phinew, const T* phin,
                               const T* phinm1, Restricted<T> r, hipStream_t st);
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
  // 3D viscoelastic: scratch for the face divergences of the weighted polymer stress (three
  // coarse arrays, written and read within launch_momentum_rhs)
  T* pol[3];
};
template <typename T>
hipError_t launch_momentum_rhs(const Dims& c, const StepConsts& k, NsIn<T> in, Restricted<T> r,
                               T* ru, T* rv, T* rw, hipStream_t st);
// Log-conformation form (lcr.hip): one RK2-TVD stage on Theta = log c,
// out = c0 * theta_n + c1 * (theta_in + dt RH(theta_in)), u fixed; with tau_out non-null also
// tau_p of the new Theta. theta_n and theta_out may alias.
template <typename T>
hipError_t launch_lcr_stage(const Dims& c, const StepConsts& k, const T* u, const T* v, const T* w,
                            const T* const theta_n[6], const T* const theta_in[6], T* const theta_out[6],
                            T* const tau_out[6], double c0, double c1, hipStream_t st);
// Both RK2-TVD stages in one pass (3D grids, central advection; polymer_rk2_fused says whether
// the grid and scheme take it): tau_out = tau^{n+1} from tau_n, u fixed; tau^(1) is not stored.
template <typename T>
bool polymer_rk2_fused(const Dims& c, const StepConsts& k);
template <typename T>
hipError_t launch_polymer_rk2(const Dims& c, const StepConsts& k, const T* u, const T* v, const T* w,
                              const T* const tau_n[6], T* const tau_out[6], hipStream_t st);
// One RK2-TVD stage: out = c0 * tau_n + c1 * (tau_in + dt RH(tau_in)), u fixed.
template <typename T>
hipError_t launch_polymer_stage(const Dims& c, const StepConsts& k, const T* u, const T* v,
                                const T* w, const T* const tau_n[6], const T* const tau_in[6],
                                T* const tau_out[6], double c0, double c1, hipStream_t st);

// ---- adjoint.hip (FP64) ----------------------------------------------------------------
// Adjoint buffers of the momentum stage (coarse; lExz, lEyz, lph_xz, lph_yz have nz + 1
// layers, the others nz).
struct AdjMomBufs {
  double *mu[3], *lph_f[3], *lG_f[3];
  double *lX, *lY, *lZ, *lExy, *lExz, *lEyz;
  double *lph_xy, *lph_xz, *lph_yz;
  double *lj[3], *J[3];
  double *lph_c, *lG_c;
};
// number of blocks of a launch3(nx, ny, nz_blocks) grid (one partial sum per block)
int adj_blocks(int nx, int ny, int nz_blocks);
// Polymer RK2 transposed: lt1, lL (9) scratch; out_tau0 += stress adjoint of tau^n; lu, lv,
// lw = lam_u^{n+1} + velocity adjoint from the polymer update. Partials: dJ/dWi, 2 regions of
// adj_blocks(nx, ny, nz).
hipError_t launch_adj_polymer(const Dims& c, const StepConsts& k, const double* u, const double* v,
                              const double* w, const double* const lam_tau[6],
                              const double* const tau_n[6], const double* const tau_1[6],
                              double* const lt1[6], double* const lL[9], double* const out_tau0[6],
                              const double* lu_in, const double* lv_in, const double* lw_in,
                              double* lu, double* lv, double* lw, double* part, hipStream_t st);
// Projection and velocity Helmholtz transposed, per Fourier mode (spec4: lam_u, lam_v, lam_w,
// lam_p on entry; lam_r (3 fields) on exit).
hipError_t launch_zpass_ns_adj(const Dims& d, const Tables<double>& tb, cx<double>* spec4,
                               const StepConsts& c, double scale, hipStream_t st);
// Momentum right-hand side transposed. lr: lam_r (3 fields of nc). Partials: dJ/dPe through
// c_j, adj_blocks(nx, ny, 3 nz).
hipError_t launch_adj_momentum(const Dims& c, const StepConsts& k, NsIn<double> in, Restricted<double> R,
                               const double* lr, const AdjMomBufs& b, double* lp_n, double* lp_nm1,
                               double* const out_tau0[6], double* const out_tau1[6], double* u0,
                               double* u1, double* v0, double* v1, double* w0, double* w1,
                               double* part, hipStream_t st);
// Restriction and chemical potential transposed: lG (fine) and the adjoint of phi^{n+1}.
hipError_t launch_adj_restrict_ch(const Dims& f, const Dims& c, const StepConsts& k, const AdjMomBufs& b,
                                  const double* lphi_new_in, double* lG, double* lphi, hipStream_t st);
// Cahn-Hilliard right-hand side and prolongation transposed. Partials: theta and Pe, each
// adj_blocks(fnx, fny, fnz).
hipError_t launch_adj_ch(const Dims& f, const Dims& c, const StepConsts& k, const double* lQ,
                         const double* lG, const double* phin, const double* phinm1,
                         const double* phinew, const double* un, const double* unm1, const double* vn,
                         const double* vnm1, const double* wn, const double* wnm1, double sin_bot,
                         double* lphi_n, double* lphi_nm1, double* u0, double* u1, double* v0,
                         double* v1, double* w0, double* w1, double* part_theta, double* part_pe,
                         hipStream_t st);
// grad3 += (sum of theta partials, Pe partials, Wi partials)
hipError_t launch_adj_final(const double* part, int n_wi, int off_pe1, int n_pe1, int off_th, int n_f,
                            int off_pe2, double* grad3, hipStream_t st);

// ---- reduce.hip -----------------------------------------------------------------------
// Writes DRPF_OBS_COUNT doubles to out_dev (device), using `partial` (device scratch of
// reduce_partials() doubles). Returns also a non-finite flag in out_dev[DRPF_OBS_COUNT].
template <typename T>
hipError_t launch_observables(const Dims& f, const Dims& c, const T* phi, const T* u, const T* v,
                              const T* w, double* partial, double* out_dev, hipStream_t st);
size_t reduce_partials();

}  // namespace drpf
