// C-ABI of the drpf library: parameter validation, scheme constants, workspace layout,
// host-built transform tables, and the per-step launch sequence (Sec. 3.2 of the paper:
// Cahn-Hilliard on the fine grid, restriction, Navier-Stokes projection, polymer stress).
#include <limits.h>
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/drpf.h"
#include "kernels.hpp"

using namespace drpf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* where) {
  return fail(DRPF_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}
#define HIPCHK(expr, where)                     \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
bool moving_walls(const drpf_params& p) {
  return p.u_wall_bottom[0] != 0.0 || p.u_wall_bottom[1] != 0.0 || p.u_wall_top[0] != 0.0 ||
         p.u_wall_top[1] != 0.0;
}
int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

Dims make_dims(int nx, int ny, int nz, double lx, double ly, double lz) {
  Dims d;
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.logx = ilog2(nx);
  d.logy = ilog2(ny);
  d.pitch = nx / 2 + 1;
  d.hx = lx / nx;
  d.hy = ly / ny;
  d.hz = lz / nz;
  d.ihx = 1.0 / d.hx;
  d.ihy = 1.0 / d.hy;
  d.ihz = 1.0 / d.hz;
  return d;
}

// Phase-field grid: refine times the flow grid in x and z, and in y for 3D grids (refine 0 is
// taken as 2, dual resolution; 1 is a single resolution).
Dims fine_dims(const drpf_params& p) {
  const int r = p.refine == 1 ? 1 : 2;
  const int ry = p.ny == 1 ? 1 : r;
  return make_dims(r * p.nx, ry * p.ny, r * p.nz, p.lx, p.ly, p.lz);
}

// Scheme constants (own derivation of the paper's formulas; see the header of this file).
StepConsts make_consts(const drpf_params& p, bool first) {
  StepConsts c;
  memset(&c, 0, sizeof(c));
  c.first = first ? 1 : 0;
  c.gamma0 = first ? 1.0 : 1.5;
  c.dt = p.dt;
  c.cn = p.cn;
  c.cn2 = p.cn * p.cn;
  c.pe = p.pe;
  // stabilisation: s_factor times the lower bound of eq. NS30 with M lambda = Cn^2 / Pe
  c.S = p.s_factor * p.cn * sqrt(4.0 * c.gamma0 * p.pe / p.dt);
  // eq. NS29: its discriminant equals 1 - 1/s_factor^2 for this S
  const double disc = 1.0 - 1.0 / (p.s_factor * p.s_factor);
  c.alpha = -(c.S / (2.0 * c.cn2)) * (1.0 + sqrt(disc));
  c.c_psi = c.alpha + c.S / c.cn2;
  const double d2r = M_PI / 180.0;
  c.cos_bot = cos(p.theta_bottom_deg * d2r);
  c.cos_top = cos(p.theta_top_deg * d2r);
  c.rho1 = 1.0;
  c.rho2 = 1.0 / p.rho_ratio;
  c.mu1 = p.viscoelastic ? p.beta : 1.0;
  c.mu2 = 1.0 / p.mu_ratio;
  c.rho0 = c.rho1 < c.rho2 ? c.rho1 : c.rho2;
  const double mumax = c.mu1 > c.mu2 ? c.mu1 : c.mu2;
  c.nu_m = mumax / (p.re * c.rho0);
  c.re = p.re;
  c.k_sigma = 3.0 / (2.0 * sqrt(2.0) * p.re * p.ca * p.cn);
  c.c_j = 0.5 * (c.rho1 - c.rho2) / p.pe;
  c.wi = p.wi;
  c.beta = p.beta;
  c.ax = p.a_ext[0];
  c.ay = p.a_ext[1];
  c.az = p.a_ext[2];
  c.inv_dt = 1.0 / p.dt;
  c.inv_cn2 = 1.0 / c.cn2;
  c.s_cn2 = c.S / c.cn2;
  c.pe_cn2 = p.pe / c.cn2;
  c.g_bot = c.cos_bot / (sqrt(2.0) * p.cn);
  c.g_top = c.cos_top / (sqrt(2.0) * p.cn);
  c.inv_re = 1.0 / p.re;
  c.inv_rho0 = 1.0 / c.rho0;
  c.inv_wi = 1.0 / p.wi;
  c.giesekus = p.giesekus_alpha;
  c.advection = p.advection;
  c.relax_kappa = p.d_w * c.gamma0 / p.dt;
  c.inv_gamma0 = 1.0 / c.gamma0;
  for (int a = 0; a < 2; ++a) {
    c.uwb[a] = p.u_wall_bottom[a];
    c.uwt[a] = p.u_wall_top[a];
  }
  return c;
}

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct TabOff {
  size_t tw_xm, tw_xn, tw_y, lam_x, lam_y, ph_x, ph_y, tw_z, tw_zq, lam_z;
};

struct Offsets {
  TabOff tf, tc;
  size_t rf, sf, rc, sc, rset[12], tau1[6], part, obs, total;
};

Offsets layout(const drpf_params& p, const Dims& F, const Dims& C) {
  const size_t es = p.precision == 32 ? 4 : 8;
  Carver cv;
  Offsets o;
  auto tabs = [&](const Dims& d, TabOff& t) {
    t.tw_xm = cv.take((size_t)(d.nx / 2) * 2 * es);
    t.tw_xn = cv.take((size_t)(d.nx / 2 + 1) * 2 * es);
    t.tw_y = cv.take((size_t)d.ny * 2 * es);
    t.lam_x = cv.take((size_t)d.pitch * 8);
    t.lam_y = cv.take((size_t)d.ny * 8);
    t.ph_x = cv.take((size_t)d.pitch * 16);
    t.ph_y = cv.take((size_t)d.ny * 16);
    t.tw_z = cv.take((size_t)d.nz * 2 * es);
    t.tw_zq = cv.take((size_t)d.nz * 2 * es);
    t.lam_z = cv.take((size_t)d.nz * 8);
  };
  tabs(F, o.tf);
  tabs(C, o.tc);
  o.rf = cv.take(F.cells() * es);
  o.sf = cv.take(F.spec() * 2 * es);
  o.rc = cv.take(3 * C.cells() * es);
  o.sc = cv.take(4 * C.spec() * 2 * es);
  const size_t nc = C.cells(), ne = (size_t)C.nx * C.ny * (C.nz + 1);
  for (int a = 0; a < 12; ++a) o.rset[a] = cv.take((a >= 10 ? ne : nc) * es);
  for (int m = 0; m < 6; ++m) o.tau1[m] = p.viscoelastic ? cv.take(nc * es) : 0;
  o.part = cv.take(reduce_partials() * 8);
  o.obs = cv.take(8 * 8);
  o.total = cv.off;
  return o;
}

}  // namespace

// Scratch of the allocation-free solve (drpf_helmholtz_solve_static): the spectral buffer
// and the right-hand side with the wall terms of one solve, for grids up to this size. Each
// GPU holds its own copy until the process ends; in host code its name is only a stand-in for
// the device address, which scratch_ptr() looks up once per device.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the first call per
// device, with that device current).
int scratch_ptr(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DRPF_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DRPF_OK;
}

}  // namespace

struct drpf_grid {
  drpf_params p;
  Dims F, C;
  StepConsts k1, k2;
  char* ws;
  Offsets o;
  // adjoint workspace (FP64 grids), attached by drpf_adjoint_attach
  char* aws = nullptr;
  // viscoelastic grids: the polymer update of a step runs on a stream of the library's own,
  // forked from the caller's stream after the velocity correction and joined before the next
  // step's momentum right-hand side (the next step's Cahn-Hilliard pass overlaps it)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool pending = false;
  // per-kernel timing: one event after each launch, one at the start of profiling
  bool prof = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kernel;
  size_t ev_used = 0;
};

namespace {

template <typename T>
Tables<T> tables(drpf_grid* g, const TabOff& t) {
  Tables<T> tb;
  tb.tw_xm = reinterpret_cast<const cx<T>*>(g->ws + t.tw_xm);
  tb.tw_xn = reinterpret_cast<const cx<T>*>(g->ws + t.tw_xn);
  tb.tw_y = reinterpret_cast<const cx<T>*>(g->ws + t.tw_y);
  tb.lam_x = reinterpret_cast<const double*>(g->ws + t.lam_x);
  tb.lam_y = reinterpret_cast<const double*>(g->ws + t.lam_y);
  tb.ph_x = reinterpret_cast<const double*>(g->ws + t.ph_x);
  tb.ph_y = reinterpret_cast<const double*>(g->ws + t.ph_y);
  tb.tw_z = reinterpret_cast<const cx<T>*>(g->ws + t.tw_z);
  tb.tw_zq = reinterpret_cast<const cx<T>*>(g->ws + t.tw_zq);
  tb.lam_z = reinterpret_cast<const double*>(g->ws + t.lam_z);
  return tb;
}

template <typename T>
Restricted<T> rset(drpf_grid* g) {
  T* a[12];
  for (int m = 0; m < 12; ++m) a[m] = reinterpret_cast<T*>(g->ws + g->o.rset[m]);
  Restricted<T> r;
  r.phi_c = a[0];
  r.G_c = a[1];
  r.G_x = a[2];
  r.G_y = a[3];
  r.G_z = a[4];
  r.ri_x = a[5];
  r.ri_y = a[6];
  r.ri_z = a[7];
  r.mu_c = a[8];
  r.mu_xy = a[9];
  r.mu_xz = a[10];
  r.mu_yz = a[11];
  return r;
}

// Host tables in long double, rounded to the storage type.
template <typename T>
int upload_tables(drpf_grid* g, const Dims& d, const TabOff& t, hipStream_t st,
                  std::vector<std::vector<unsigned char>>& keep) {
  const long double pi = 3.141592653589793238462643383279502884L;
  auto put = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    keep.emplace_back((const unsigned char*)src, (const unsigned char*)src + bytes);
    return hipMemcpyAsync(g->ws + off, keep.back().data(), bytes, hipMemcpyHostToDevice, st);
  };
  std::vector<T> tw;
  const int M = d.nx / 2;
  tw.resize(2 * M);
  for (int i = 0; i < M; ++i) {
    tw[2 * i] = (T)cosl(2 * pi * i / M);
    tw[2 * i + 1] = (T)-sinl(2 * pi * i / M);
  }
  HIPCHK(put(t.tw_xm, tw.data(), tw.size() * sizeof(T)), "upload twiddles");
  tw.assign(2 * (M + 1), 0);
  for (int k = 0; k <= M; ++k) {
    tw[2 * k] = (T)cosl(2 * pi * k / d.nx);
    tw[2 * k + 1] = (T)-sinl(2 * pi * k / d.nx);
  }
  HIPCHK(put(t.tw_xn, tw.data(), tw.size() * sizeof(T)), "upload twiddles");
  tw.assign(2 * d.ny, 0);
  for (int i = 0; i < d.ny; ++i) {
    tw[2 * i] = (T)cosl(2 * pi * i / d.ny);
    tw[2 * i + 1] = (T)-sinl(2 * pi * i / d.ny);
  }
  HIPCHK(put(t.tw_y, tw.data(), tw.size() * sizeof(T)), "upload twiddles");
  std::vector<double> lx(d.pitch), ly(d.ny), px(2 * d.pitch), py(2 * d.ny);
  for (int k = 0; k < d.pitch; ++k) {
    const double s = sin(M_PI * k / d.nx);
    lx[k] = -4.0 / (d.hx * d.hx) * s * s;
    px[2 * k] = (double)cosl(2 * pi * k / d.nx);
    px[2 * k + 1] = (double)sinl(2 * pi * k / d.nx);
  }
  for (int k = 0; k < d.ny; ++k) {
    const double s = sin(M_PI * k / d.ny);
    ly[k] = -4.0 / (d.hy * d.hy) * s * s;
    py[2 * k] = (double)cosl(2 * pi * k / d.ny);
    py[2 * k + 1] = (double)sinl(2 * pi * k / d.ny);
  }
  HIPCHK(put(t.lam_x, lx.data(), lx.size() * 8), "upload eigenvalues");
  HIPCHK(put(t.lam_y, ly.data(), ly.size() * 8), "upload eigenvalues");
  HIPCHK(put(t.ph_x, px.data(), px.size() * 8), "upload phases");
  HIPCHK(put(t.ph_y, py.data(), py.size() * 8), "upload phases");
  tw.assign(2 * d.nz, 0);
  for (int i = 0; i < d.nz; ++i) {
    tw[2 * i] = (T)cosl(2 * pi * i / d.nz);
    tw[2 * i + 1] = (T)-sinl(2 * pi * i / d.nz);
  }
  HIPCHK(put(t.tw_z, tw.data(), tw.size() * sizeof(T)), "upload twiddles");
  for (int m = 0; m < d.nz; ++m) {
    tw[2 * m] = (T)cosl(pi * m / (2 * d.nz));
    tw[2 * m + 1] = (T)-sinl(pi * m / (2 * d.nz));
  }
  HIPCHK(put(t.tw_zq, tw.data(), tw.size() * sizeof(T)), "upload twiddles");
  std::vector<double> lz(d.nz);
  for (int m = 0; m < d.nz; ++m) {
    const double s = sin(M_PI * m / (2.0 * d.nz));
    lz[m] = -4.0 / (d.hz * d.hz) * s * s;
  }
  HIPCHK(put(t.lam_z, lz.data(), lz.size() * 8), "upload eigenvalues");
  return DRPF_OK;
}

const char* const kKernelNames[DRPF_NKERNELS] = {
    "ch_rhs", "fft_x_fwd_fine", "fft_y_fwd_fine", "zpass_ch", "fft_y_inv_fine", "fft_x_inv_fine",
    "restrict_g", "momentum_rhs", "fft_x_fwd_coarse", "fft_y_fwd_coarse", "zpass_ns",
    "fft_y_inv_coarse", "fft_x_inv_coarse", "polymer_stage1", "polymer_stage2", "weno_adv_fine",
    "fft_xy_fwd_coarse", "fft_xy_inv_coarse", "polymer_rk2"};

void mark(drpf_grid* g, int kernel, hipStream_t st) {
  if (!g->prof || g->ev_used >= g->ev.size()) return;
  // a failed record shows up as an error of drpf_profile_end's elapsed-time query
  (void)hipEventRecord(g->ev[g->ev_used], st);
  g->ev_kernel[g->ev_used] = kernel;
  ++g->ev_used;
}

// Pointers of one step: the two input levels of every field, and where the step writes its
// results. The outputs may alias the n-1 inputs (u, v, w, p, tau): each output is written only
// after the last read of that input.
template <typename T>
struct StepIO {
  const T *phin, *phinm1;
  T* phinew;
  const T *un, *unm1, *vn, *vnm1, *wn, *wnm1, *pn, *pnm1;
  T *uo, *vo, *wo, *po;
  const T* taun[6];
  const T* taunm1[6];
  T* tauo[6];
  T* theta[6];  // log-conformation, level n in, level n+1 out (constitutive 1)
};

// One coupled step (Sec. 3.2): Cahn-Hilliard, restriction, Navier-Stokes, polymer stress.
// Leaves the restricted coarse set and the first polymer stage in the workspace.
template <typename T>
int step_one(drpf_grid* g, const StepIO<T>& io, const StepConsts& K, hipStream_t st, bool overlap = false) {
  const Dims& F = g->F;
  const Dims& C = g->C;
  const Tables<T> tf = tables<T>(g, g->o.tf), tc = tables<T>(g, g->o.tc);
  T* Rf = reinterpret_cast<T*>(g->ws + g->o.rf);
  cx<T>* Sf = reinterpret_cast<cx<T>*>(g->ws + g->o.sf);
  T* Rc = reinterpret_cast<T*>(g->ws + g->o.rc);
  cx<T>* Sc = reinterpret_cast<cx<T>*>(g->ws + g->o.sc);
  const Restricted<T> R = rset<T>(g);
  const size_t nc = C.cells();
  const bool ve = g->p.viscoelastic != 0;
  // ---- Cahn-Hilliard on the fine grid
  ChIn<T> ci{io.phin, io.phinm1, io.un, io.unm1, io.vn, io.vnm1, io.wn, io.wnm1, nullptr};
  if (g->p.advection == 1) {
    // WENO-Z advection first, into the fine spectral buffer (free until the transform)
    T* adv = reinterpret_cast<T*>(Sf);
    HIPCHK(launch_weno_adv_fine<T>(F, C, K, ci, adv, st), "weno advection");
    mark(g, 15, st);
    ci.adv = adv;
  }
  HIPCHK(launch_ch_rhs<T>(F, C, K, ci, Rf, st), "ch_rhs");
  mark(g, 0, st);
  const T* inf[4] = {Rf, nullptr, nullptr, nullptr};
  HIPCHK(launch_fft_x_fwd<T>(F, tf, inf, 1, Sf, st), "fft_x fine");
  mark(g, 1, st);
  HIPCHK(launch_fft_y<T>(F, tf, Sf, 1, false, st), "fft_y fine");
  mark(g, 2, st);
  HIPCHK(launch_zpass_ch<T>(F, tf, Sf, K.c_psi, K.alpha, 1.0 / ((double)F.nx * F.ny),
                            -K.relax_kappa / F.hz, st),
         "zpass_ch");
  mark(g, 3, st);
  HIPCHK(launch_fft_y<T>(F, tf, Sf, 1, true, st), "ifft_y fine");
  mark(g, 4, st);
  RealSet<T> of;
  memset(&of, 0, sizeof(of));
  of.p[0] = io.phinew;
  of.nfields = 1;
  HIPCHK(launch_fft_x_inv<T>(F, tf, Sf, of, st), "ifft_x fine");
  mark(g, 5, st);
  // ---- restriction, chemical potential, properties
  if (g->p.refine == 1)
    HIPCHK(launch_props_single<T>(C, K, io.phinew, io.phin, io.phinm1, R, st), "props_single");
  else
    HIPCHK(launch_restrict_g<T>(F, C, K, io.phinew, io.phin, io.phinm1, R, st), "restrict_g");
  mark(g, 6, st);
  // ---- Navier-Stokes on the coarse grid
  NsIn<T> ni;
  ni.un = io.un;
  ni.unm1 = io.unm1;
  ni.vn = io.vn;
  ni.vnm1 = io.vnm1;
  ni.wn = io.wn;
  ni.wnm1 = io.wnm1;
  ni.pn = io.pn;
  ni.pnm1 = io.pnm1;
  for (int m = 0; m < 6; ++m) {
    ni.taun[m] = ve ? io.taun[m] : nullptr;
    ni.taunm1[m] = ve ? io.taunm1[m] : nullptr;
  }
  ni.viscoelastic = ve ? 1 : 0;
  // the first three stage-1 polymer arrays are free until the polymer update
  for (int a = 0; a < 3; ++a) ni.pol[a] = ve ? reinterpret_cast<T*>(g->ws + g->o.tau1[a]) : nullptr;
  // the previous step's polymer update (tau^n here, and the stage arrays) must be complete
  if (g->pending) {
    HIPCHK(hipStreamWaitEvent(st, g->ev_join, 0), "join polymer stream");
    g->pending = false;
  }
  HIPCHK(launch_momentum_rhs<T>(C, K, ni, R, Rc, Rc + nc, Rc + 2 * nc, st), "momentum_rhs");
  mark(g, 7, st);
  const T* inc[4] = {Rc, Rc + nc, Rc + 2 * nc, nullptr};
  // a coarse layer that fits in one block's LDS takes the x and y passes in one kernel
  const bool fused = fft_xy_fits<T>(C);
  if (fused) {
    HIPCHK(launch_fft_xy_fwd<T>(C, tc, inc, 3, Sc, st), "fft_xy coarse");
    mark(g, 16, st);
  } else {
    HIPCHK(launch_fft_x_fwd<T>(C, tc, inc, 3, Sc, st), "fft_x coarse");
    mark(g, 8, st);
    HIPCHK(launch_fft_y<T>(C, tc, Sc, 3, false, st), "fft_y coarse");
    mark(g, 9, st);
  }
  HIPCHK(launch_zpass_ns<T>(C, tc, Sc, K, 1.0 / ((double)C.nx * C.ny), st), "zpass_ns");
  mark(g, 10, st);
  RealSet<T> oc;
  memset(&oc, 0, sizeof(oc));
  oc.p[0] = io.uo;
  oc.p[1] = io.vo;
  oc.p[2] = io.wo;
  oc.p[3] = io.po;
  oc.add[3] = io.pn;
  oc.nfields = 4;
  if (fused) {
    HIPCHK(launch_fft_xy_inv<T>(C, tc, Sc, oc, st), "ifft_xy coarse");
    mark(g, 17, st);
  } else {
    HIPCHK(launch_fft_y<T>(C, tc, Sc, 4, true, st), "ifft_y coarse");
    mark(g, 11, st);
    HIPCHK(launch_fft_x_inv<T>(C, tc, Sc, oc, st), "ifft_x coarse");
    mark(g, 12, st);
  }
  // ---- polymer stress, RK2-TVD with u^{n+1}: on the library's stream when overlapping (it reads
  // u^{n+1} and tau^n and writes tau^{n+1} and the stage arrays, none of which the next step's
  // Cahn-Hilliard pass and restriction touch)
  hipStream_t pst = st;
  if (ve && overlap) {
    HIPCHK(hipEventRecord(g->ev_fork, st), "fork polymer stream");
    HIPCHK(hipStreamWaitEvent(g->side, g->ev_fork, 0), "fork polymer stream");
    pst = g->side;
  }
  if (ve) {
    T* t1[6];
    const T* t1c[6];
    for (int m = 0; m < 6; ++m) {
      t1[m] = reinterpret_cast<T*>(g->ws + g->o.tau1[m]);
      t1c[m] = t1[m];
    }
    if (g->p.constitutive == 1) {
      // log-conformation (eqs. NS42-NS46): Theta^(1) in the stage buffer, Theta^{n+1} in place,
      // then tau^{n+1} from it
      const T* thn[6];
      for (int m = 0; m < 6; ++m) thn[m] = io.theta[m];
      HIPCHK(launch_lcr_stage<T>(C, K, io.uo, io.vo, io.wo, thn, thn, t1, nullptr, 0.0, 1.0, pst),
             "log-conformation stage 1");
      mark(g, 13, pst);
      HIPCHK(launch_lcr_stage<T>(C, K, io.uo, io.vo, io.wo, thn, t1c, io.theta, io.tauo, 0.5, 0.5, pst),
             "log-conformation stage 2");
      mark(g, 14, pst);
    } else if (polymer_rk2_fused<T>(C, K)) {
      // both stages in one pass; tau^(1) is not stored
      HIPCHK(launch_polymer_rk2<T>(C, K, io.uo, io.vo, io.wo, io.taun, io.tauo, pst), "polymer RK2");
      mark(g, 18, pst);
    } else {
      HIPCHK(launch_polymer_stage<T>(C, K, io.uo, io.vo, io.wo, io.taun, io.taun, t1, 0.0, 1.0, pst),
             "polymer stage 1");
      mark(g, 13, pst);
      HIPCHK(launch_polymer_stage<T>(C, K, io.uo, io.vo, io.wo, io.taun, t1c, io.tauo, 0.5, 0.5, pst),
             "polymer stage 2");
      mark(g, 14, pst);
    }
  }
  if (ve && overlap) {
    HIPCHK(hipEventRecord(g->ev_join, g->side), "join polymer stream");
    g->pending = true;
  }
  return DRPF_OK;
}

template <typename T>
StepIO<T> state_io(const drpf_state* s) {
  StepIO<T> io;
  io.phin = (const T*)s->phi[0];
  io.phinm1 = (const T*)s->phi[1];
  io.phinew = (T*)s->phi[2];
  io.un = (const T*)s->u[0];
  io.unm1 = (const T*)s->u[1];
  io.vn = (const T*)s->v[0];
  io.vnm1 = (const T*)s->v[1];
  io.wn = (const T*)s->w[0];
  io.wnm1 = (const T*)s->w[1];
  io.pn = (const T*)s->p[0];
  io.pnm1 = (const T*)s->p[1];
  io.uo = (T*)s->u[1];
  io.vo = (T*)s->v[1];
  io.wo = (T*)s->w[1];
  io.po = (T*)s->p[1];
  for (int m = 0; m < 6; ++m) {
    io.taun[m] = (const T*)s->tau[0][m];
    io.taunm1[m] = (const T*)s->tau[1][m];
    io.tauo[m] = (T*)s->tau[1][m];
    io.theta[m] = (T*)s->theta[m];
  }
  return io;
}

// Finiteness of the phase field (count of non-finite values) and of the velocities (their
// kinetic-energy sum) of level n of s, from the observables reduction; synchronises st.
template <typename T>
int check_finite(drpf_grid* g, const drpf_state* s, hipStream_t st) {
  double* part = reinterpret_cast<double*>(g->ws + g->o.part);
  double* obs = reinterpret_cast<double*>(g->ws + g->o.obs);
  HIPCHK(launch_observables<T>(g->F, g->C, (const T*)s->phi[0], (const T*)s->u[0], (const T*)s->v[0],
                               (const T*)s->w[0], part, obs, st),
         "finite check");
  double host[6];
  HIPCHK(hipMemcpyAsync(host, obs, 6 * sizeof(double), hipMemcpyDeviceToHost, st), "copy finite check");
  HIPCHK(hipStreamSynchronize(st), "synchronise finite check");
  if (host[5] != 0.0 || !isfinite(host[3]))
    return fail(DRPF_ENONFINITE, "non-finite " + std::string(host[5] != 0.0 ? "phase field" : "velocity") +
                                     " after step " + std::to_string(s->step));
  return DRPF_OK;
}

template <typename T>
int step_impl(drpf_grid* g, drpf_state* s, int nsteps, hipStream_t st) {
  const bool ve = g->p.viscoelastic != 0;
  const int every = g->p.check_finite_every;
  // the polymer update overlaps the next step on the library's stream, except while per-kernel
  // events are being recorded (they time one stream)
  const bool overlap = g->side != nullptr && !g->prof;
  // whatever happens, the caller's stream ends up after the last polymer update
  struct Join {
    drpf_grid* g;
    hipStream_t st;
    ~Join() {
      if (g->pending) {
        (void)hipStreamWaitEvent(st, g->ev_join, 0);
        g->pending = false;
      }
    }
  } join{g, st};
  for (int n = 0; n < nsteps; ++n) {
    const StepConsts& K = s->step == 0 ? g->k1 : g->k2;
    const int rc = step_one<T>(g, state_io<T>(s), K, st, overlap);
    if (rc) return rc;
    // ---- rotate time levels (pointer swaps only)
    void* ph0 = s->phi[0];
    void* ph1 = s->phi[1];
    s->phi[0] = s->phi[2];
    s->phi[1] = ph0;
    s->phi[2] = ph1;
    void* tmp;
    tmp = s->u[0]; s->u[0] = s->u[1]; s->u[1] = tmp;
    tmp = s->v[0]; s->v[0] = s->v[1]; s->v[1] = tmp;
    tmp = s->w[0]; s->w[0] = s->w[1]; s->w[1] = tmp;
    tmp = s->p[0]; s->p[0] = s->p[1]; s->p[1] = tmp;
    if (ve)
      for (int m = 0; m < 6; ++m) {
        tmp = s->tau[0][m];
        s->tau[0][m] = s->tau[1][m];
        s->tau[1][m] = tmp;
      }
    s->step += 1;
    if (every > 0 && s->step % every == 0) {
      const int cf = check_finite<T>(g, s, st);
      if (cf) return cf;
    }
  }
  return DRPF_OK;
}

// The solve's scratch: the spectral buffer S and the buffer R of the right-hand side with the
// wall terms (used only with wall data); by default the grid's workspace buffers.
template <typename T>
int helmholtz_impl(drpf_grid* g, int which, int bc, double coeff, double shift, const void* rhs,
                   const void* wall, void* x, hipStream_t st, void* s_scr = nullptr,
                   void* r_scr = nullptr) {
  const Dims& d = which == DRPF_GRID_FINE ? g->F : g->C;
  const Tables<T> tb = tables<T>(g, which == DRPF_GRID_FINE ? g->o.tf : g->o.tc);
  cx<T>* S = s_scr ? reinterpret_cast<cx<T>*>(s_scr)
                   : reinterpret_cast<cx<T>*>(g->ws + (which == DRPF_GRID_FINE ? g->o.sf : g->o.sc));
  const T* in[4] = {(const T*)rhs, nullptr, nullptr, nullptr};
  if (wall) {
    // the known wall terms move to the right-hand side: rhs - coeff b into the right-hand-side
    // buffer, which the transforms then read
    T* R = r_scr ? reinterpret_cast<T*>(r_scr)
                 : reinterpret_cast<T*>(g->ws + (which == DRPF_GRID_FINE ? g->o.rf : g->o.rc));
    HIPCHK(launch_wall_rhs<T>(d, bc, coeff, (const T*)rhs, (const T*)wall, R, st), "wall data");
    in[0] = R;
  }
  HIPCHK(launch_fft_x_fwd<T>(d, tb, in, 1, S, st), "fft_x");
  HIPCHK(launch_fft_y<T>(d, tb, S, 1, false, st), "fft_y");
  HIPCHK(launch_zpass_helmholtz<T>(d, tb, S, bc, coeff, shift, 1.0 / ((double)d.nx * d.ny), st),
         "zpass");
  HIPCHK(launch_fft_y<T>(d, tb, S, 1, true, st), "ifft_y");
  RealSet<T> o;
  memset(&o, 0, sizeof(o));
  o.p[0] = (T*)x;
  o.nfields = 1;
  HIPCHK(launch_fft_x_inv<T>(d, tb, S, o, st), "ifft_x");
  if (wall && bc == DRPF_BC_FACE_DIRICHLET)
    HIPCHK(launch_top_layer<T>(d, (const T*)wall + (size_t)d.nx * d.ny, (T*)x, st), "top wall layer");
  return DRPF_OK;
}

template <typename T>
int observables_impl(drpf_grid* g, const drpf_state* s, double* out, int n, hipStream_t st) {
  double* part = reinterpret_cast<double*>(g->ws + g->o.part);
  double* obs = reinterpret_cast<double*>(g->ws + g->o.obs);
  HIPCHK(launch_observables<T>(g->F, g->C, (const T*)s->phi[0], (const T*)s->u[0],
                               (const T*)s->v[0], (const T*)s->w[0], part, obs, st),
         "observables");
  double host[8];
  HIPCHK(hipMemcpyAsync(host, obs, 6 * sizeof(double), hipMemcpyDeviceToHost, st), "copy observables");
  HIPCHK(hipStreamSynchronize(st), "synchronise");
  const int m = n < DRPF_OBS_COUNT ? n : DRPF_OBS_COUNT;
  for (int i = 0; i < m; ++i) out[i] = host[i];
  if (host[5] != 0.0) return fail(DRPF_ENONFINITE, "phase field holds non-finite values");
  return DRPF_OK;
}

// Adjoint workspace: forward intermediates of the recomputed step, then the adjoint stage
// buffers (FP64).
struct AdjLayout {
  size_t phinew, lG, lQ;                                     // fine
  size_t unew, vnew, wnew, pnew, taunew[6], lt1[6], lL[9], lu[3];
  size_t mu[3], lph_f[3], lG_f[3], lX, lY, lZ, lExy, lph_xy, lj[3], J[3], lph_c, lG_c;
  size_t lExz, lEyz, lph_xz, lph_yz;                         // nz + 1 layers
  size_t part;
  int nbA, nbM, nbF;
  size_t total;
};

AdjLayout adj_layout(const Dims& F, const Dims& C) {
  Carver cv;
  AdjLayout a;
  const size_t nf = F.cells() * 8, nc = C.cells() * 8, ne = (size_t)C.nx * C.ny * (C.nz + 1) * 8;
  a.phinew = cv.take(nf);
  a.lG = cv.take(nf);
  a.lQ = cv.take(nf);
  a.unew = cv.take(nc);
  a.vnew = cv.take(nc);
  a.wnew = cv.take(nc);
  a.pnew = cv.take(nc);
  for (int m = 0; m < 6; ++m) a.taunew[m] = cv.take(nc);
  for (int m = 0; m < 6; ++m) a.lt1[m] = cv.take(nc);
  for (int m = 0; m < 9; ++m) a.lL[m] = cv.take(nc);
  for (int m = 0; m < 3; ++m) a.lu[m] = cv.take(nc);
  for (int m = 0; m < 3; ++m) a.mu[m] = cv.take(nc);
  for (int m = 0; m < 3; ++m) a.lph_f[m] = cv.take(nc);
  for (int m = 0; m < 3; ++m) a.lG_f[m] = cv.take(nc);
  a.lX = cv.take(nc);
  a.lY = cv.take(nc);
  a.lZ = cv.take(nc);
  a.lExy = cv.take(nc);
  a.lph_xy = cv.take(nc);
  for (int m = 0; m < 3; ++m) a.lj[m] = cv.take(nc);
  for (int m = 0; m < 3; ++m) a.J[m] = cv.take(nc);
  a.lph_c = cv.take(nc);
  a.lG_c = cv.take(nc);
  a.lExz = cv.take(ne);
  a.lEyz = cv.take(ne);
  a.lph_xz = cv.take(ne);
  a.lph_yz = cv.take(ne);
  a.nbA = adj_blocks(C.nx, C.ny, C.nz);
  a.nbM = adj_blocks(C.nx, C.ny, 3 * C.nz);
  a.nbF = adj_blocks(F.nx, F.ny, F.nz);
  a.part = cv.take((size_t)(2 * a.nbA + a.nbM + 2 * a.nbF) * 8);
  a.total = cv.off;
  return a;
}

int adjoint_impl(drpf_grid* g, const drpf_state* x, const drpf_state* xn, drpf_adj* lam, double* d_grad3,
                 hipStream_t st) {
  using T = double;
  const Dims& F = g->F;
  const Dims& C = g->C;
  const StepConsts& K = x->step == 0 ? g->k1 : g->k2;
  const bool ve = g->p.viscoelastic != 0;
  const AdjLayout A = adj_layout(F, C);
  auto P = [&](size_t off) { return reinterpret_cast<T*>(g->aws + off); };
  const Tables<T> tf = tables<T>(g, g->o.tf), tc = tables<T>(g, g->o.tc);
  T* Rc = reinterpret_cast<T*>(g->ws + g->o.rc);
  cx<T>* Sc = reinterpret_cast<cx<T>*>(g->ws + g->o.sc);
  cx<T>* Sf = reinterpret_cast<cx<T>*>(g->ws + g->o.sf);
  const size_t nc = C.cells();
  // ---- forward intermediates: with the state after the step given, only the restricted
  // coarse set and the first polymer stage are recomputed; otherwise the whole step is,
  // into the adjoint workspace
  StepIO<T> io = state_io<T>(x);
  if (xn) {
    io.phinew = (T*)xn->phi[0];
    io.uo = (T*)xn->u[0];
    io.vo = (T*)xn->v[0];
    io.wo = (T*)xn->w[0];
    io.po = (T*)xn->p[0];
    HIPCHK(launch_restrict_g<T>(F, C, K, io.phinew, io.phin, io.phinm1, rset<T>(g), st), "adjoint restrict_g");
    if (ve) {
      T* t1[6];
      for (int m = 0; m < 6; ++m) t1[m] = reinterpret_cast<T*>(g->ws + g->o.tau1[m]);
      HIPCHK(launch_polymer_stage<T>(C, K, io.uo, io.vo, io.wo, io.taun, io.taun, t1, 0.0, 1.0, st),
             "adjoint polymer stage 1");
    }
  } else {
    io.phinew = P(A.phinew);
    io.uo = P(A.unew);
    io.vo = P(A.vnew);
    io.wo = P(A.wnew);
    io.po = P(A.pnew);
    for (int m = 0; m < 6; ++m) io.tauo[m] = P(A.taunew[m]);
    const int rc = step_one<T>(g, io, K, st);
    if (rc) return rc;
    if (ve && polymer_rk2_fused<T>(C, K)) {
      // the fused forward update keeps no first stage: recompute it for the transposed update
      T* t1[6];
      for (int m = 0; m < 6; ++m) t1[m] = reinterpret_cast<T*>(g->ws + g->o.tau1[m]);
      HIPCHK(launch_polymer_stage<T>(C, K, io.uo, io.vo, io.wo, io.taun, io.taun, t1, 0.0, 1.0, st),
             "adjoint polymer stage 1");
    }
  }
  double* part = P(A.part);
  // ---- polymer
  const T* lu_use[3] = {(const T*)lam->u[0], (const T*)lam->v[0], (const T*)lam->w[0]};
  if (ve) {
    const T* lt[6];
    const T* tn[6];
    const T* t1[6];
    T* l1[6];
    T* lL[9];
    T* ot0[6];
    for (int m = 0; m < 6; ++m) {
      lt[m] = (const T*)lam->tau[0][m];
      tn[m] = (const T*)x->tau[0][m];
      t1[m] = reinterpret_cast<const T*>(g->ws + g->o.tau1[m]);
      l1[m] = P(A.lt1[m]);
      ot0[m] = (T*)lam->tau[1][m];
    }
    for (int m = 0; m < 9; ++m) lL[m] = P(A.lL[m]);
    HIPCHK(launch_adj_polymer(C, K, io.uo, io.vo, io.wo, lt, tn, t1, l1, lL, ot0, lu_use[0],
                              lu_use[1], lu_use[2], P(A.lu[0]), P(A.lu[1]), P(A.lu[2]), part, st),
           "adjoint polymer");
    for (int a = 0; a < 3; ++a) lu_use[a] = P(A.lu[a]);
  }
  // ---- projection and velocity Helmholtz, transposed
  HIPCHK(launch_fft_x_fwd<T>(C, tc, lu_use, 3, Sc, st), "adjoint fft_x coarse");
  const T* lpin[4] = {(const T*)lam->p[0], nullptr, nullptr, nullptr};
  HIPCHK(launch_fft_x_fwd<T>(C, tc, lpin, 1, Sc + 3 * C.spec(), st), "adjoint fft_x coarse p");
  HIPCHK(launch_fft_y<T>(C, tc, Sc, 4, false, st), "adjoint fft_y coarse");
  HIPCHK(launch_zpass_ns_adj(C, tc, Sc, K, 1.0 / ((double)C.nx * C.ny), st), "adjoint zpass_ns");
  HIPCHK(launch_fft_y<T>(C, tc, Sc, 3, true, st), "adjoint ifft_y coarse");
  RealSet<T> oc;
  memset(&oc, 0, sizeof(oc));
  oc.p[0] = Rc;
  oc.p[1] = Rc + nc;
  oc.p[2] = Rc + 2 * nc;
  oc.nfields = 3;
  HIPCHK(launch_fft_x_inv<T>(C, tc, Sc, oc, st), "adjoint ifft_x coarse");
  // ---- momentum right-hand side, transposed
  NsIn<T> ni;
  ni.un = io.un;
  ni.unm1 = io.unm1;
  ni.vn = io.vn;
  ni.vnm1 = io.vnm1;
  ni.wn = io.wn;
  ni.wnm1 = io.wnm1;
  ni.pn = io.pn;
  ni.pnm1 = io.pnm1;
  for (int m = 0; m < 6; ++m) {
    ni.taun[m] = ve ? io.taun[m] : nullptr;
    ni.taunm1[m] = ve ? io.taunm1[m] : nullptr;
  }
  ni.viscoelastic = ve ? 1 : 0;
  AdjMomBufs b;
  for (int a = 0; a < 3; ++a) {
    b.mu[a] = P(A.mu[a]);
    b.lph_f[a] = P(A.lph_f[a]);
    b.lG_f[a] = P(A.lG_f[a]);
    b.lj[a] = P(A.lj[a]);
    b.J[a] = P(A.J[a]);
  }
  b.lX = P(A.lX);
  b.lY = P(A.lY);
  b.lZ = P(A.lZ);
  b.lExy = P(A.lExy);
  b.lExz = P(A.lExz);
  b.lEyz = P(A.lEyz);
  b.lph_xy = P(A.lph_xy);
  b.lph_xz = P(A.lph_xz);
  b.lph_yz = P(A.lph_yz);
  b.lph_c = P(A.lph_c);
  b.lG_c = P(A.lG_c);
  T* ot0[6];
  T* ot1[6];
  for (int m = 0; m < 6; ++m) {
    ot0[m] = ve ? (T*)lam->tau[1][m] : nullptr;
    ot1[m] = ve ? (T*)lam->tau[0][m] : nullptr;
  }
  T* const u0 = (T*)lam->u[1];
  T* const u1 = (T*)lam->u[0];
  T* const v0 = (T*)lam->v[1];
  T* const v1 = (T*)lam->v[0];
  T* const w0 = (T*)lam->w[1];
  T* const w1 = (T*)lam->w[0];
  HIPCHK(launch_adj_momentum(C, K, ni, rset<T>(g), Rc, b, (T*)lam->p[1], (T*)lam->p[0], ot0, ot1, u0, u1, v0,
                             v1, w0, w1, part + 2 * A.nbA, st),
         "adjoint momentum");
  // ---- restriction and chemical potential, transposed; then the fused CH solve
  HIPCHK(launch_adj_restrict_ch(F, C, K, b, (const T*)lam->phi[0], P(A.lG), P(A.lQ), st), "adjoint restrict");
  const T* inf[4] = {P(A.lQ), nullptr, nullptr, nullptr};
  HIPCHK(launch_fft_x_fwd<T>(F, tf, inf, 1, Sf, st), "adjoint fft_x fine");
  HIPCHK(launch_fft_y<T>(F, tf, Sf, 1, false, st), "adjoint fft_y fine");
  // the fused Cahn-Hilliard operator is symmetric with static walls; with relaxed walls its
  // rank-two wall term is not, and the transposed pass solves with the transpose
  HIPCHK(launch_zpass_ch<T>(F, tf, Sf, K.c_psi, K.alpha, 1.0 / ((double)F.nx * F.ny), -K.relax_kappa / F.hz, st,
                            K.relax_kappa != 0.0),
         "adjoint zpass_ch");
  HIPCHK(launch_fft_y<T>(F, tf, Sf, 1, true, st), "adjoint ifft_y fine");
  RealSet<T> of;
  memset(&of, 0, sizeof(of));
  of.p[0] = P(A.lQ);
  of.nfields = 1;
  HIPCHK(launch_fft_x_inv<T>(F, tf, Sf, of, st), "adjoint ifft_x fine");
  const double sin_bot = sin(g->p.theta_bottom_deg * M_PI / 180.0);
  const int off_th = 2 * A.nbA + A.nbM, off_pe2 = off_th + A.nbF;
  HIPCHK(launch_adj_ch(F, C, K, P(A.lQ), P(A.lG), io.phin, io.phinm1, io.phinew, io.un, io.unm1, io.vn,
                       io.vnm1, io.wn, io.wnm1, sin_bot, (T*)lam->phi[1], (T*)lam->phi[0], u0, u1, v0, v1, w0,
                       w1, part + off_th, part + off_pe2, st),
         "adjoint Cahn-Hilliard");
  HIPCHK(launch_adj_final(part, ve ? 2 * A.nbA : 0, 2 * A.nbA, A.nbM, off_th, A.nbF, off_pe2, d_grad3, st),
         "adjoint gradient sums");
  // ---- the adjoint of level n was accumulated in the [1] buffers, that of n-1 in [0]
  auto swap = [](void*& a, void*& b2) {
    void* t = a;
    a = b2;
    b2 = t;
  };
  swap(lam->phi[0], lam->phi[1]);
  swap(lam->u[0], lam->u[1]);
  swap(lam->v[0], lam->v[1]);
  swap(lam->w[0], lam->w[1]);
  swap(lam->p[0], lam->p[1]);
  if (ve)
    for (int m = 0; m < 6; ++m) swap(lam->tau[0][m], lam->tau[1][m]);
  return DRPF_OK;
}

}  // namespace

extern "C" {

const char* drpf_last_error(void) { return g_err.c_str(); }

int drpf_params_default(drpf_params* p) {
  if (!p) return fail(DRPF_EINVAL, "null params");
  memset(p, 0, sizeof(*p));
  p->nx = 64;
  p->ny = 1;
  p->nz = 32;
  p->lx = 2.0;
  p->ly = 2.0 / 64;
  p->lz = 1.0;
  p->re = 10.0;
  p->ca = 0.1;
  p->cn = 0.01;
  p->pe = 1000.0;
  p->wi = 1.0;
  p->beta = 1.0;
  p->theta_bottom_deg = 60.0;
  p->theta_top_deg = 90.0;
  p->rho_ratio = 1.0;
  p->mu_ratio = 1.0;
  p->dt = 1e-4;
  p->s_factor = 1.0;
  p->viscoelastic = 0;
  p->precision = 64;
  p->refine = 2;
  return DRPF_OK;
}

int drpf_validate(const drpf_params* p) {
  if (!p) return fail(DRPF_EINVAL, "null params");
  if (!pow2(p->nx) || p->nx < 4 || p->nx > 1024) return fail(DRPF_EINVAL, "nx must be a power of two in [4, 1024]");
  // the wall-normal solve keeps a whole fine column (2 nz rows) in one thread block
  if (!pow2(p->nz) || p->nz < 4 || p->nz > 512) return fail(DRPF_EINVAL, "nz must be a power of two in [4, 512]");
  if (!(p->ny == 1 || (pow2(p->ny) && p->ny >= 4 && p->ny <= 1024)))
    return fail(DRPF_EINVAL, "ny must be 1 or a power of two in [4, 1024]");
  if (!(p->lx > 0 && p->ly > 0 && p->lz > 0)) return fail(DRPF_EINVAL, "box lengths must be > 0");
  if (!(p->re > 0 && p->ca > 0 && p->cn > 0 && p->pe > 0 && p->dt > 0))
    return fail(DRPF_EINVAL, "Re, Ca, Cn, Pe and dt must be > 0");
  if (!(p->s_factor >= 1.0)) return fail(DRPF_EINVAL, "s_factor must be >= 1 (eq. NS30)");
  if (!(p->theta_bottom_deg >= 0 && p->theta_bottom_deg <= 180 && p->theta_top_deg >= 0 &&
        p->theta_top_deg <= 180))
    return fail(DRPF_EINVAL, "contact angles must lie in [0, 180] degrees");
  if (!(p->rho_ratio > 0 && p->mu_ratio > 0)) return fail(DRPF_EINVAL, "density and viscosity ratios must be > 0");
  if (p->viscoelastic && !(p->wi > 0 && p->beta > 0 && p->beta <= 1))
    return fail(DRPF_EINVAL, "viscoelastic drop needs Wi > 0 and beta in (0, 1]");
  if (!(p->constitutive == 0 || p->constitutive == 1)) return fail(DRPF_EINVAL, "constitutive must be 0 or 1");
  if (!(p->refine == 0 || p->refine == 1 || p->refine == 2)) return fail(DRPF_EINVAL, "refine must be 1 or 2");
  if (!(p->advection == 0 || p->advection == 1)) return fail(DRPF_EINVAL, "advection must be 0 or 1");
  if (!(p->d_w >= 0.0 && p->d_w < 1e30)) return fail(DRPF_EINVAL, "d_w must be finite and >= 0");
  if (p->constitutive == 1 && !p->viscoelastic)
    return fail(DRPF_EINVAL, "the log-conformation form needs viscoelastic");
  if (!(p->giesekus_alpha >= 0 && p->giesekus_alpha <= 0.5))
    return fail(DRPF_EINVAL, "giesekus_alpha must lie in [0, 0.5]");
  if (p->giesekus_alpha > 0 && !(p->viscoelastic && p->beta < 1))
    return fail(DRPF_EINVAL, "a Giesekus term needs viscoelastic and beta < 1");
  if (!(p->precision == 64 || p->precision == 32)) return fail(DRPF_EINVAL, "precision must be 64 or 32");
  for (int a = 0; a < 3; ++a)
    if (!isfinite(p->a_ext[a])) return fail(DRPF_EINVAL, "a_ext must be finite");
  for (int a = 0; a < 2; ++a)
    if (!isfinite(p->u_wall_bottom[a]) || !isfinite(p->u_wall_top[a]))
      return fail(DRPF_EINVAL, "wall velocities must be finite");
  if (p->check_finite_every < 0) return fail(DRPF_EINVAL, "check_finite_every must be >= 0");
  return DRPF_OK;
}

int drpf_field_elems(const drpf_params* p, size_t* fine, size_t* coarse) {
  const int rc = drpf_validate(p);
  if (rc) return rc;
  if (!fine || !coarse) return fail(DRPF_EINVAL, "null output");
  *fine = fine_dims(*p).cells();
  *coarse = (size_t)p->nx * p->ny * p->nz;
  return DRPF_OK;
}

int drpf_workspace_bytes(const drpf_params* p, size_t* bytes) {
  const int rc = drpf_validate(p);
  if (rc) return rc;
  if (!bytes) return fail(DRPF_EINVAL, "null output");
  const Dims F = fine_dims(*p);
  const Dims C = make_dims(p->nx, p->ny, p->nz, p->lx, p->ly, p->lz);
  *bytes = layout(*p, F, C).total;
  return DRPF_OK;
}

int drpf_init_grid(const drpf_params* p, void* d_workspace, size_t bytes, void* stream,
                   drpf_grid** out) {
  int rc = drpf_validate(p);
  if (rc) return rc;
  if (!out) return fail(DRPF_EINVAL, "null output handle");
  size_t need = 0;
  drpf_workspace_bytes(p, &need);
  if (!d_workspace) return fail(DRPF_EWORKSPACE, "null workspace");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(DRPF_EWORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < need)
    return fail(DRPF_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  drpf_grid* g = new drpf_grid;
  g->p = *p;
  g->F = fine_dims(*p);
  g->C = make_dims(p->nx, p->ny, p->nz, p->lx, p->ly, p->lz);
  g->k1 = make_consts(*p, true);
  g->k2 = make_consts(*p, false);
  g->ws = (char*)d_workspace;
  g->o = layout(*p, g->F, g->C);
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<unsigned char>> keep;
  if (p->precision == 64) {
    rc = upload_tables<double>(g, g->F, g->o.tf, st, keep);
    if (!rc) rc = upload_tables<double>(g, g->C, g->o.tc, st, keep);
  } else {
    rc = upload_tables<float>(g, g->F, g->o.tf, st, keep);
    if (!rc) rc = upload_tables<float>(g, g->C, g->o.tc, st, keep);
  }
  if (!rc) {
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = hip_fail(e, "init synchronise");
  }
  if (!rc) {
    // set-up of the allocation-free solve on this device
    void* scr = nullptr;
    rc = scratch_ptr(&scr);
  }
  if (!rc && p->viscoelastic) {
    // the stream the polymer update overlaps on (default priority) and its fork/join events
    hipError_t e = hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) rc = hip_fail(e, "polymer stream");
  }
  if (rc) {
    drpf_destroy(g);
    return rc;
  }
  *out = g;
  return DRPF_OK;
}

int drpf_destroy(drpf_grid* g) {
  if (g) {
    for (auto e : g->ev) (void)hipEventDestroy(e);
    if (g->side) {
      (void)hipStreamSynchronize(g->side);
      (void)hipStreamDestroy(g->side);
    }
    if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
    if (g->ev_join) (void)hipEventDestroy(g->ev_join);
  }
  delete g;
  return DRPF_OK;
}

int drpf_state_layout(const drpf_grid* g, drpf_layout* out) {
  if (!g || !out) return fail(DRPF_EINVAL, "null grid or output");
  memset(out, 0, sizeof(*out));
  out->elem_bytes = g->p.precision == 32 ? 4 : 8;
  // origin offsets in cells: centres at +1/2, a component's own faces at +1
  const double ctr[3] = {0.5, 0.5, 0.5};
  const double fx[3] = {1.0, 0.5, 0.5}, fy[3] = {0.5, 1.0, 0.5}, fz[3] = {0.5, 0.5, 1.0};
  const int ve = g->p.viscoelastic != 0, lcr = g->p.constitutive == 1;
  struct Spec {
    const Dims* d;
    const double* off;
    int arrays;
  } spec[DRPF_NFIELDS] = {{&g->F, ctr, 3}, {&g->C, fx, 2}, {&g->C, fy, 2}, {&g->C, fz, 2},
                          {&g->C, ctr, 2}, {&g->C, ctr, ve ? 12 : 0}, {&g->C, ctr, lcr ? 6 : 0}};
  size_t total = 0;
  for (int f = 0; f < DRPF_NFIELDS; ++f) {
    drpf_field_layout& L = out->field[f];
    const Dims& d = *spec[f].d;
    L.n[0] = d.nx;
    L.n[1] = d.ny;
    L.n[2] = d.nz;
    L.stride[0] = 1;
    L.stride[1] = (size_t)d.nx;
    L.stride[2] = (size_t)d.nx * d.ny;
    L.elems = d.cells();
    L.arrays = spec[f].arrays;
    const double h[3] = {d.hx, d.hy, d.hz};
    for (int a = 0; a < 3; ++a) {
      L.spacing[a] = h[a];
      L.origin[a] = spec[f].off[a] * h[a];
    }
    total += (size_t)L.arrays * L.elems * out->elem_bytes;
  }
  out->state_bytes = total;
  return DRPF_OK;
}

int drpf_step(drpf_grid* g, drpf_state* s, int nsteps, void* stream) {
  if (!g || !s) return fail(DRPF_EINVAL, "null grid or state");
  if (nsteps < 0) return fail(DRPF_EINVAL, "nsteps must be >= 0");
  if (!s->phi[0] || !s->phi[1] || !s->phi[2] || !s->u[0] || !s->u[1] || !s->v[0] || !s->v[1] ||
      !s->w[0] || !s->w[1] || !s->p[0] || !s->p[1])
    return fail(DRPF_EINVAL, "null state pointer");
  if (g->p.viscoelastic)
    for (int l = 0; l < 2; ++l)
      for (int m = 0; m < 6; ++m)
        if (!s->tau[l][m]) return fail(DRPF_EINVAL, "null polymer stress pointer");
  if (g->p.constitutive == 1)
    for (int m = 0; m < 6; ++m)
      if (!s->theta[m]) return fail(DRPF_EINVAL, "null log-conformation pointer");
  if (s->step < 0) return fail(DRPF_EINVAL, "negative step counter");
  hipStream_t st = (hipStream_t)stream;
  return g->p.precision == 64 ? step_impl<double>(g, s, nsteps, st) : step_impl<float>(g, s, nsteps, st);
}

int drpf_prolong(drpf_grid* g, const void* u, const void* v, const void* w, void* uf, void* vf,
                 void* wf, void* stream) {
  if (!g || !u || !v || !w || !uf || !vf || !wf) return fail(DRPF_EINVAL, "null argument");
  if (g->p.refine == 1) return fail(DRPF_EUNSUPPORTED, "no dual grid: single resolution");
  hipStream_t st = (hipStream_t)stream;
  if (g->p.precision == 64)
    HIPCHK(launch_prolong<double>(g->F, g->C, (const double*)u, (const double*)v, (const double*)w,
                                  (double*)uf, (double*)vf, (double*)wf, st),
           "prolong");
  else
    HIPCHK(launch_prolong<float>(g->F, g->C, (const float*)u, (const float*)v, (const float*)w,
                                 (float*)uf, (float*)vf, (float*)wf, st),
           "prolong");
  return DRPF_OK;
}

int drpf_restrict(drpf_grid* g, const void* fine, void* coarse, int location, void* stream) {
  if (!g || !fine || !coarse) return fail(DRPF_EINVAL, "null argument");
  if (g->p.refine == 1) return fail(DRPF_EUNSUPPORTED, "no dual grid: single resolution");
  if (location < DRPF_CENTER || location > DRPF_EDGE_YZ) return fail(DRPF_EINVAL, "bad location");
  hipStream_t st = (hipStream_t)stream;
  if (g->p.precision == 64)
    HIPCHK(launch_restrict<double>(g->F, g->C, (const double*)fine, (double*)coarse, location, st),
           "restrict");
  else
    HIPCHK(launch_restrict<float>(g->F, g->C, (const float*)fine, (float*)coarse, location, st),
           "restrict");
  return DRPF_OK;
}

static int helmholtz_args(drpf_grid* g, int which_grid, int bc, double coeff, double shift, const void* rhs,
                          void* x) {
  if (!g || !rhs || !x) return fail(DRPF_EINVAL, "null argument");
  if (which_grid != DRPF_GRID_FINE && which_grid != DRPF_GRID_COARSE) return fail(DRPF_EINVAL, "bad grid");
  if (bc < DRPF_BC_NEUMANN || bc > DRPF_BC_FACE_DIRICHLET) return fail(DRPF_EINVAL, "bad boundary kind");
  if (!(coeff > 0) || !(shift >= 0) || !isfinite(coeff) || !isfinite(shift))
    return fail(DRPF_EINVAL, "need coeff > 0 and shift >= 0");
  if (shift == 0 && bc != DRPF_BC_NEUMANN) return fail(DRPF_EINVAL, "shift 0 only with Neumann walls");
  return DRPF_OK;
}

int drpf_helmholtz_solve_static(drpf_grid* g, int which_grid, int bc, double coeff, double shift,
                                const void* rhs, const void* wall_data, void* x, void* stream) {
  const int rc = helmholtz_args(g, which_grid, bc, coeff, shift, rhs, x);
  if (rc) return rc;
  const Dims& d = which_grid == DRPF_GRID_FINE ? g->F : g->C;
  const size_t es = g->p.precision == 32 ? 4 : 8;
  const size_t sbytes = (d.spec() * 2 * es + 255) & ~(size_t)255;
  const size_t need = sbytes + (wall_data ? d.cells() * es : 0);
  if (need > kStaticScratchBytes)
    return fail(DRPF_EWORKSPACE, "drpf_helmholtz_solve_static: the solve needs " + std::to_string(need) +
                                     " bytes of scratch, above the static limit of " +
                                     std::to_string(kStaticScratchBytes));
  void* scr = nullptr;
  const int pc = scratch_ptr(&scr);
  if (pc) return pc;
  char* base = (char*)scr;
  hipStream_t st = (hipStream_t)stream;
  return g->p.precision == 64
             ? helmholtz_impl<double>(g, which_grid, bc, coeff, shift, rhs, wall_data, x, st, base, base + sbytes)
             : helmholtz_impl<float>(g, which_grid, bc, coeff, shift, rhs, wall_data, x, st, base, base + sbytes);
}

int drpf_helmholtz_solve(drpf_grid* g, int which_grid, int bc, double coeff, double shift,
                         const void* rhs, const void* wall_data, void* x, void* stream) {
  const int rc = helmholtz_args(g, which_grid, bc, coeff, shift, rhs, x);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  return g->p.precision == 64 ? helmholtz_impl<double>(g, which_grid, bc, coeff, shift, rhs, wall_data, x, st)
                              : helmholtz_impl<float>(g, which_grid, bc, coeff, shift, rhs, wall_data, x, st);
}

int drpf_observables(drpf_grid* g, const drpf_state* s, double* out, int n, void* stream) {
  if (!g || !s || !out || n < 0) return fail(DRPF_EINVAL, "null argument");
  if (!s->phi[0] || !s->u[0] || !s->v[0] || !s->w[0]) return fail(DRPF_EINVAL, "null state pointer");
  hipStream_t st = (hipStream_t)stream;
  return g->p.precision == 64 ? observables_impl<double>(g, s, out, n, st)
                              : observables_impl<float>(g, s, out, n, st);
}

int drpf_profile_begin(drpf_grid* g, int max_launches, void* stream) {
  if (!g || max_launches < 1) return fail(DRPF_EINVAL, "need a grid and max_launches >= 1");
  if (g->prof) return fail(DRPF_EINVAL, "profiling already active");
  g->ev.assign((size_t)max_launches + 1, nullptr);
  g->ev_kernel.assign((size_t)max_launches + 1, -1);
  for (auto& e : g->ev) HIPCHK(hipEventCreate(&e), "event create");
  g->prof = true;
  g->ev_used = 0;
  mark(g, -1, (hipStream_t)stream);
  return DRPF_OK;
}

int drpf_profile_end(drpf_grid* g, double* total_ms, int* launches, int n) {
  if (!g || !g->prof) return fail(DRPF_EINVAL, "profiling not active");
  int rc = DRPF_OK;
  if (g->ev_used > 0) {
    const hipError_t e = hipEventSynchronize(g->ev[g->ev_used - 1]);
    if (e != hipSuccess) rc = hip_fail(e, "event synchronise");
  }
  for (int k = 0; k < n; ++k) {
    if (total_ms) total_ms[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  for (size_t a = 1; rc == DRPF_OK && a < g->ev_used; ++a) {
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, g->ev[a - 1], g->ev[a]);
    if (e != hipSuccess) {
      rc = hip_fail(e, "event elapsed time");
      break;
    }
    const int k = g->ev_kernel[a];
    if (k >= 0 && k < n) {
      if (total_ms) total_ms[k] += ms;
      if (launches) launches[k] += 1;
    }
  }
  for (auto e : g->ev) (void)hipEventDestroy(e);
  g->ev.clear();
  g->ev_kernel.clear();
  g->ev_used = 0;
  g->prof = false;
  return rc;
}

const char* drpf_kernel_name(int id) {
  return (id >= 0 && id < DRPF_NKERNELS) ? kKernelNames[id] : "";
}

int drpf_debug_field(drpf_grid* g, int id, void** ptr, size_t* count) {
  if (!g || !ptr || !count) return fail(DRPF_EINVAL, "null argument");
  const size_t nc = g->C.cells(), ne = (size_t)g->C.nx * g->C.ny * (g->C.nz + 1);
  const size_t es = g->p.precision == 32 ? 4 : 8;
  if (id >= 0 && id < 12) {
    *ptr = g->ws + g->o.rset[id];
    *count = id >= 10 ? ne : nc;
    return DRPF_OK;
  }
  if (id >= 12 && id < 15) {
    *ptr = g->ws + g->o.rc + (size_t)(id - 12) * nc * es;
    *count = nc;
    return DRPF_OK;
  }
  return fail(DRPF_EINVAL, "unknown debug field id");
}

int drpf_adjoint_workspace_bytes(const drpf_params* p, size_t* bytes) {
  const int rc = drpf_validate(p);
  if (rc) return rc;
  if (!bytes) return fail(DRPF_EINVAL, "null output");
  if (p->precision != 64) return fail(DRPF_EUNSUPPORTED, "the adjoint runs on FP64 grids only");
  if (p->constitutive != 0)
    return fail(DRPF_EUNSUPPORTED, "the adjoint covers the stress form only (Oldroyd-B or Giesekus)");
  if (p->d_w > 0.0 && moving_walls(*p))
    return fail(DRPF_EUNSUPPORTED, "the adjoint covers relaxed walls (d_w > 0) at rest only");
  if (p->refine == 1) return fail(DRPF_EUNSUPPORTED, "the adjoint covers the dual-resolution step only");
  const Dims F = fine_dims(*p);
  // the transposed fine-grid kernels index a fine field with 32-bit integers
  if (F.cells() > (size_t)INT_MAX)
    return fail(DRPF_EUNSUPPORTED, "the adjoint needs a phase-field grid of at most 2^31 - 1 cells");
  const Dims C = make_dims(p->nx, p->ny, p->nz, p->lx, p->ly, p->lz);
  *bytes = adj_layout(F, C).total;
  return DRPF_OK;
}

int drpf_adjoint_attach(drpf_grid* g, void* d_workspace, size_t bytes) {
  if (!g) return fail(DRPF_EINVAL, "null grid");
  if (g->p.precision != 64) return fail(DRPF_EUNSUPPORTED, "the adjoint runs on FP64 grids only");
  if (g->p.constitutive != 0)
    return fail(DRPF_EUNSUPPORTED, "the adjoint covers the stress form only (Oldroyd-B or Giesekus)");
  if (g->p.d_w > 0.0 && moving_walls(g->p))
    return fail(DRPF_EUNSUPPORTED, "the adjoint covers relaxed walls (d_w > 0) at rest only");
  if (g->p.refine == 1) return fail(DRPF_EUNSUPPORTED, "the adjoint covers the dual-resolution step only");
  if (!d_workspace) return fail(DRPF_EWORKSPACE, "null adjoint workspace");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(DRPF_EWORKSPACE, "adjoint workspace must be 256-byte aligned");
  const size_t need = adj_layout(g->F, g->C).total;
  if (bytes < need)
    return fail(DRPF_EWORKSPACE, "adjoint workspace too small: need " + std::to_string(need) + " bytes");
  g->aws = (char*)d_workspace;
  return DRPF_OK;
}

int drpf_adjoint_step(drpf_grid* g, const drpf_state* x, const drpf_state* x_next, drpf_adj* lam,
                      double* d_grad3, void* stream) {
  if (!g || !x || !lam || !d_grad3) return fail(DRPF_EINVAL, "null argument");
  if (g->p.precision != 64) return fail(DRPF_EUNSUPPORTED, "the adjoint runs on FP64 grids only");
  if (g->p.constitutive != 0)
    return fail(DRPF_EUNSUPPORTED, "the adjoint covers the stress form only (Oldroyd-B or Giesekus)");
  if (g->p.d_w > 0.0 && moving_walls(g->p))
    return fail(DRPF_EUNSUPPORTED, "the adjoint covers relaxed walls (d_w > 0) at rest only");
  if (g->p.refine == 1) return fail(DRPF_EUNSUPPORTED, "the adjoint covers the dual-resolution step only");
  if (!g->aws) return fail(DRPF_EINVAL, "no adjoint workspace attached");
  if (!x->phi[0] || !x->phi[1] || !x->u[0] || !x->u[1] || !x->v[0] || !x->v[1] || !x->w[0] || !x->w[1] ||
      !x->p[0] || !x->p[1])
    return fail(DRPF_EINVAL, "null state pointer");
  for (int l = 0; l < 2; ++l)
    if (!lam->phi[l] || !lam->u[l] || !lam->v[l] || !lam->w[l] || !lam->p[l])
      return fail(DRPF_EINVAL, "null adjoint pointer");
  if (g->p.viscoelastic)
    for (int l = 0; l < 2; ++l)
      for (int m = 0; m < 6; ++m)
        if (!x->tau[l][m] || !lam->tau[l][m]) return fail(DRPF_EINVAL, "null polymer stress pointer");
  if (x->step < 0) return fail(DRPF_EINVAL, "negative step counter");
  if (x_next) {
    if (!x_next->phi[0] || !x_next->u[0] || !x_next->v[0] || !x_next->w[0] || !x_next->p[0])
      return fail(DRPF_EINVAL, "null pointer in the state after the step");
    if (x_next->step != x->step + 1) return fail(DRPF_EINVAL, "x_next must be the state one step after x_n");
  }
  return adjoint_impl(g, x, x_next, lam, d_grad3, (hipStream_t)stream);
}

}  // extern "C"
