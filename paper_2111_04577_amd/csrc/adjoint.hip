// Discrete adjoint of one coupled step (FP64): the transpose of the step's Jacobian applied to
// the adjoint of the state after the step, taken stage by stage in reverse order of Sec. 3.2:
//
//   polymer    -- the two stages of the RK2-TVD update (eqs. NS42, NS44) transposed: the
//                 stress adjoint through the advection, the upper-convected coupling and the
//                 relaxation, and the velocity adjoint through the velocity gradient and the
//                 advecting velocity (adj_polymer_s2, adj_polymer_s1, adj_polymer_vel);
//   projection -- the correction and pressure-increment Poisson solve transposed, then the
//                 velocity Helmholtz solves (symmetric operators: the same spectral solves),
//                 in the wall-normal pass of tridiag.hip;
//   momentum   -- every term of the right-hand side of eq. NS36 transposed: faces
//                 (adj_mom_faces: face-local factors and the adjoints of 1/rho and G at
//                 faces), stress-like adjoints at centres and edges, the diffusive-flux
//                 adjoint and the pressure levels (adj_stress), the centred quantities
//                 (adj_centre: polymer stress, phi, G), and the velocity levels
//                 (adj_mom_vel);
//   transfer   -- the restriction of eq. dual2 transposed (every coarse location scatters
//                 back onto the fine cells it averaged) together with the chemical potential
//                 (adj_restrict_ch); the prolongation of eq. dual1 transposed (adj_prolong);
//   Cahn-Hilliard -- the fused Dong solve is symmetric: its transpose is the same spectral
//                 pass; the right-hand side Q of eq. NS28, the wetting data and the advection
//                 are transposed in adj_ch.
//
// Gradients with respect to the bottom static angle, Pe and Wi are accumulated from per-block
// partial sums in a fixed order. Every formula is the exact transpose of the forward kernels'
// arithmetic (coarse.hpp, fine.hpp, stencil_ch.hip), ghost rules included: a transposed
// difference with odd ghosts uses even ghosts and the reverse.
#include "coarse.hpp"
#include "fine.hpp"
#include "weno.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;
using D = double;

// Per-block partial sum in a fixed order (deterministic).
__device__ void block_partial(D v, D* part) {
  __shared__ D sh[kBlock];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nt = blockDim.x * blockDim.y;
  sh[tid] = v;
  __syncthreads();
  if (tid == 0) {
    D s = 0;
    for (int t = 0; t < nt; ++t) s += sh[t];
    part[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
  __syncthreads();  // sh is reused by a following call
}

struct Six {
  const D* p[6];
};
struct SixOut {
  D* p[6];
};
struct Nine {
  D* p[9];
};

__device__ __forceinline__ void cell_index(int& k, int& j, int& i) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  i = bx * blockDim.x + threadIdx.x;
  j = by * blockDim.y + threadIdx.y;
  k = bz;
}

// ---- WENO-Z advection transposed (advection 1, Sec. 3.2.3) ---------------------------------
// The face value of weno_face (stencil v[0..4] = the five upwind cells, the face between v[2]
// and v[3]) and its gradient g = d value / d v. value = sum a_k q_k / sum a_k, so
// d value = sum (a_k dq_k + (q_k - value) da_k) / sum a_k, da_k = d_k (dt5 / (b_k + eps) -
// t5 db_k / (b_k + eps)^2), t5 = |b_0 - b_2| with dt5 = sign(b_0 - b_2)(db_0 - db_2), taken as
// 0 at a tie (the subgradient of |x| at 0 that reverse-mode differentiation takes).
__device__ D weno_face_grad(const D v[5], D g[5]) {
  const D eps = 1e-40;
  const D a = v[0], b = v[1], c = v[2], d = v[3], e = v[4];
  const D q[3] = {(2 * a - 7 * b + 11 * c) / 6, (-b + 5 * c + 2 * d) / 6, (2 * c + 5 * d - e) / 6};
  const D dq[3][5] = {{2.0 / 6, -7.0 / 6, 11.0 / 6, 0, 0}, {0, -1.0 / 6, 5.0 / 6, 2.0 / 6, 0}, {0, 0, 2.0 / 6, 5.0 / 6, -1.0 / 6}};
  const D s0 = a - 2 * b + c, r0 = a - 4 * b + 3 * c;
  const D s1 = b - 2 * c + d, r1 = b - d;
  const D s2 = c - 2 * d + e, r2 = 3 * c - 4 * d + e;
  const D c13 = 13.0 / 12.0;
  const D bt[3] = {c13 * s0 * s0 + 0.25 * r0 * r0, c13 * s1 * s1 + 0.25 * r1 * r1, c13 * s2 * s2 + 0.25 * r2 * r2};
  // d beta_k / d v: 13/6 s_k (second-difference row) + 1/2 r_k (one-sided row)
  const D db[3][5] = {{2 * c13 * s0 + 0.5 * r0, -4 * c13 * s0 - 2.0 * r0, 2 * c13 * s0 + 1.5 * r0, 0, 0},
                      {0, 2 * c13 * s1 + 0.5 * r1, -4 * c13 * s1, 2 * c13 * s1 - 0.5 * r1, 0},
                      {0, 0, 2 * c13 * s2 + 1.5 * r2, -4 * c13 * s2 - 2.0 * r2, 2 * c13 * s2 + 0.5 * r2}};
  const D dk[3] = {0.1, 0.6, 0.3};
  const D diff = bt[0] - bt[2];
  const D t5 = fabs(diff), sg = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
  D w[3], al[3], S = 0, num = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w[k] = 1.0 / (bt[k] + eps);
    al[k] = dk[k] * (1.0 + t5 * w[k]);
    S += al[k];
    num += al[k] * q[k];
  }
  const D val = num / S;
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    const D dt5 = sg * (db[0][p] - db[2][p]);
    D acc = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const D dal = dk[k] * (dt5 * w[k] - t5 * w[k] * w[k] * db[k][p]);
      acc += al[k] * dq[k][p] + (q[k] - val) * dal;
    }
    g[p] = acc / S;
  }
  return val;
}

// The five stencil cells, in weno_face's order, of the face between cells f and f + 1 along an
// axis of n cells: from cell f's side for a positive face velocity, from f + 1's otherwise;
// periodic (PER) or mirrored beyond the walls
template <bool PER>
__device__ __forceinline__ void weno_cells(int f, int n, bool pos, int c[5]) {
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    const int cc = pos ? f - 2 + p : f + 3 - p;
    c[p] = PER ? wrap(cc, n) : mirror_index(cc, n);
  }
}

// Transposed WENO-Z flux divergence along one axis, gathered at cell j: the sum over the faces
// f (between cells f and f + 1) whose upwind stencil holds cell j of lF(f) u(f) d(face
// value)/d(q_j). Periodic axes (n a power of two) visit each face once also when n < 6; on a
// walled axis only the faces 0 .. n - 2 carry flux. q(c), u(f), lF(f) take in-range indices.
template <bool PER, typename Q, typename U, typename LF>
__device__ D weno_adj_axis(int j, int n, Q&& q, U&& u, LF&& lF) {
  D s = 0;
  const int nf = PER && n < 6 ? n : 6;
  for (int o = 0; o < nf; ++o) {
    int f = j - 3 + o;
    if (PER)
      f = wrap(f, n);
    else if (f < 0 || f > n - 2)
      continue;
    const D uf = u(f);
    int c[5];
    weno_cells<PER>(f, n, uf > 0.0, c);
    bool hit = false;
#pragma unroll
    for (int p = 0; p < 5; ++p) hit = hit || c[p] == j;
    if (!hit) continue;
    D v[5], g[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) v[p] = q(c[p]);
    weno_face_grad(v, g);
    D acc = 0;
#pragma unroll
    for (int p = 0; p < 5; ++p) acc += c[p] == j ? g[p] : 0.0;
    s += lF(f) * uf * acc;
  }
  return s;
}

// WENO-Z value at the face between cells f and f + 1 (upwind side by the face velocity uf)
template <bool PER, typename Q>
__device__ __forceinline__ D weno_value(int f, int n, D uf, Q&& q) {
  int c[5];
  weno_cells<PER>(f, n, uf > 0.0, c);
  return weno_face<D>(q(c[0]), q(c[1]), q(c[2]), q(c[3]), q(c[4]));
}

// Transposed stress right-hand side for fixed velocity: out = (d RH / d tau)^T g, per cell.
// Advection -div(u tau) with face-mean stress (or, WENO, the WENO-Z face value of the stage's
// input stress tq, which the transpose depends on) and zero wall flux; upper-convected
// coupling L_ca tau_cb + tau_ac L_cb; relaxation -tau / Wi; the Giesekus term -gk tau.tau
// (tqc: the cell's input stress).
template <bool WENO>
__device__ __forceinline__ void rh_tau_T(const Six& g, const Six& tq, int k, int j, int i, int nx, int ny,
                                         int nz, const Coarse<D>& U, const Coarse<D>& V, const Coarse<D>& W,
                                         D uxp, D uxm, D vyp, D vym, D wzp, D wzm, D ihx, D ihy, D ihz,
                                         D inv_wi, const D L[3][3], const D gc[6], const D tqc[6], D gk,
                                         D out[6]) {
  const D h = 0.5;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const Coarse<D> G{g.p[m], nx, ny, nz};
    const D g0 = gc[m];
    D adv;
    if (!WENO) {
      const D gzp = k < nz - 1 ? G.at(k + 1, j, i) : 0.0;
      const D gzm = k > 0 ? G.at(k - 1, j, i) : 0.0;
      adv = (h * uxp * (G.at(k, j, i + 1) - g0) + h * uxm * (g0 - G.at(k, j, i - 1))) * ihx +
            (h * vyp * (G.at(k, j + 1, i) - g0) + h * vym * (g0 - G.at(k, j - 1, i))) * ihy +
            (h * wzp * (gzp - g0) + h * wzm * (g0 - gzm)) * ihz;
    } else {
      // RH = -div(F): the face between cells f and f + 1 carries (g_{f+1} - g_f) / h
      const Coarse<D> Q{tq.p[m], nx, ny, nz};
      adv = weno_adj_axis<true>(
          i, nx, [&](int c) { return Q.at(k, j, c); }, [&](int f) { return U.at(k, j, f); },
          [&](int f) { return (G.at(k, j, f + 1) - G.at(k, j, f)) * ihx; });
      adv += weno_adj_axis<true>(
          j, ny, [&](int c) { return Q.at(k, c, i); }, [&](int f) { return V.at(k, f, i); },
          [&](int f) { return (G.at(k, f + 1, i) - G.at(k, f, i)) * ihy; });
      adv += weno_adj_axis<false>(
          k, nz, [&](int c) { return Q.at(c, j, i); }, [&](int f) { return W.at(f, j, i); },
          [&](int f) { return (G.at(f + 1, j, i) - G.at(f, j, i)) * ihz; });
    }
    out[m] = adv - g0 * inv_wi;
  }
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int a = pairs[m][0], b = pairs[m][1];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out[tidx(c, b)] += L[c][a] * gc[m];
      out[tidx(a, c)] += L[c][b] * gc[m];
      // (tau.tau)_ab = sum_c tau_ac tau_cb
      out[tidx(a, c)] -= gk * gc[m] * tqc[tidx(c, b)];
      out[tidx(c, b)] -= gk * gc[m] * tqc[tidx(a, c)];
    }
  }
}

// sum over components of -g_ab ((1 - beta)(L_ab + L_ba) - tau_ab), the Wi-derivative of the
// relaxation term times Wi^2
__device__ __forceinline__ D wi_term(const D g[6], const D tau[6], const D L[3][3], D omb) {
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  D s = 0;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int a = pairs[m][0], b = pairs[m][1];
    s -= g[m] * (omb * (L[a][b] + L[b][a]) - tau[m]);
  }
  return s;
}

struct PolyArgs {
  const D *u, *v, *w;  // u^{n+1}
  int nx, ny, nz;
  D ihx, ihy, ihz, dt, inv_wi, omb;
  D gk;  // Giesekus: alpha / (1 - beta), 0 for Oldroyd-B
  Walls<D> wl;  // tangential wall velocities (eq. NS13) for the forward velocity gradient
};

// ---- polymer, second stage: lt1 = 0.5 lam + 0.5 dt RH_tau^T lam ----------------------------
template <bool WENO>
__global__ void __launch_bounds__(kBlock)
    k_adj_polymer_s2(PolyArgs a, Six lam, Six t1, SixOut lt1, D* part) {
  int k, j, i;
  cell_index(k, j, i);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int id = (k * ny + j) * nx + i;
  const Coarse<D> U{a.u, nx, ny, nz}, V{a.v, nx, ny, nz}, W{a.w, nx, ny, nz};
  D L[3][3];
  velocity_gradient(U, V, W, k, j, i, nz, a.ihx, a.ihy, a.ihz, L, a.wl);
  const D uxp = U.at(k, j, i), uxm = U.at(k, j, i - 1), vyp = V.at(k, j, i), vym = V.at(k, j - 1, i);
  const D wzp = k < nz - 1 ? W.at(k, j, i) : 0.0, wzm = k > 0 ? W.at(k - 1, j, i) : 0.0;
  D gc[6], tc[6], out[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    gc[m] = lam.p[m][id];
    tc[m] = t1.p[m][id];
  }
  rh_tau_T<WENO>(lam, t1, k, j, i, nx, ny, nz, U, V, W, uxp, uxm, vyp, vym, wzp, wzm, a.ihx, a.ihy, a.ihz,
                 a.inv_wi, L, gc, tc, a.gk, out);
#pragma unroll
  for (int m = 0; m < 6; ++m) lt1.p[m][id] = 0.5 * gc[m] + 0.5 * a.dt * out[m];
  block_partial(0.5 * a.dt * wi_term(gc, tc, L, a.omb) * a.inv_wi * a.inv_wi, part);
}

// ---- polymer, first stage: lam_tau^n += 0.5 lam + lt1 + dt RH_tau^T lt1; velocity-gradient
// adjoint of both stages ----------------------------------------------------------------------
template <bool WENO>
__global__ void __launch_bounds__(kBlock)
    k_adj_polymer_s1(PolyArgs a, Six lam, Six lt1, Six tn, Six t1, SixOut out_tau0, Nine lL, D* part) {
  int k, j, i;
  cell_index(k, j, i);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int id = (k * ny + j) * nx + i;
  const Coarse<D> U{a.u, nx, ny, nz}, V{a.v, nx, ny, nz}, W{a.w, nx, ny, nz};
  D L[3][3];
  velocity_gradient(U, V, W, k, j, i, nz, a.ihx, a.ihy, a.ihz, L, a.wl);
  const D uxp = U.at(k, j, i), uxm = U.at(k, j, i - 1), vyp = V.at(k, j, i), vym = V.at(k, j - 1, i);
  const D wzp = k < nz - 1 ? W.at(k, j, i) : 0.0, wzm = k > 0 ? W.at(k - 1, j, i) : 0.0;
  D lc[6], gc[6], tnc[6], t1c[6], out[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    lc[m] = lam.p[m][id];
    gc[m] = lt1.p[m][id];
    tnc[m] = tn.p[m][id];
    t1c[m] = t1.p[m][id];
  }
  rh_tau_T<WENO>(lt1, tn, k, j, i, nx, ny, nz, U, V, W, uxp, uxm, vyp, vym, wzp, wzm, a.ihx, a.ihy, a.ihz,
                 a.inv_wi, L, gc, tnc, a.gk, out);
#pragma unroll
  for (int m = 0; m < 6; ++m) out_tau0.p[m][id] += 0.5 * lc[m] + gc[m] + a.dt * out[m];
  // adjoint of L from both stages: weights 0.5 dt (lam with t1) and dt (lt1 with tau^n)
  D G[3][3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) G[p][q] = 0;
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int aa = pairs[m][0], b = pairs[m][1];
    const D w2 = 0.5 * a.dt * lc[m], w1 = a.dt * gc[m];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      G[c][aa] += w2 * t1c[tidx(c, b)] + w1 * tnc[tidx(c, b)];
      G[c][b] += w2 * t1c[tidx(aa, c)] + w1 * tnc[tidx(aa, c)];
    }
    const D r = a.omb * a.inv_wi * (w2 + w1);
    G[aa][b] += r;
    G[b][aa] += r;
  }
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) lL.p[3 * p + q][id] = G[p][q];
  block_partial(a.dt * wi_term(gc, tnc, L, a.omb) * a.inv_wi * a.inv_wi, part);
}

// ---- polymer, velocity adjoint: lam_u^{n+1} plus the transposed velocity gradient and the
// advecting-velocity part of both stages -----------------------------------------------------
template <bool WENO>
__global__ void __launch_bounds__(kBlock)
    k_adj_polymer_vel(PolyArgs a, const D* __restrict__ lu_in, const D* __restrict__ lv_in,
                      const D* __restrict__ lw_in, Six lam, Six lt1, Six tn, Six t1, Nine lL,
                      D* __restrict__ lu, D* __restrict__ lv, D* __restrict__ lw) {
  int k, j, i;
  cell_index(k, j, i);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int id = (k * ny + j) * nx + i;
  const D h = 0.5;
  auto LL = [&](int c, int kk, int jj, int ii) -> D {
    return lL.p[c][(min(max(kk, 0), nz - 1) * ny + wrap(jj, ny)) * nx + wrap(ii, nx)];
  };
  // the advecting-velocity part at the face between cells p0 and p1 (along axis ax: 0 x, 1 y,
  // 2 z): the face value of each stage's input stress times the jump of that stage's adjoint
  const Coarse<D> Uc{a.u, nx, ny, nz}, Vc{a.v, nx, ny, nz}, Wc{a.w, nx, ny, nz};
  auto adv = [&](int i0, int j0, int k0, int i1, int j1, int k1, int ax) -> D {
    const int p0 = (k0 * ny + wrap(j0, ny)) * nx + wrap(i0, nx);
    const int p1 = (k1 * ny + wrap(j1, ny)) * nx + wrap(i1, nx);
    D s = 0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      D f1, fn;
      if (!WENO) {
        f1 = h * (t1.p[m][p0] + t1.p[m][p1]);
        fn = h * (tn.p[m][p0] + tn.p[m][p1]);
      } else {
        const Coarse<D> T1{t1.p[m], nx, ny, nz}, TN{tn.p[m], nx, ny, nz};
        if (ax == 0) {
          const D uf = Uc.at(k0, j0, i0);
          f1 = weno_value<true>(wrap(i0, nx), nx, uf, [&](int c) { return T1.at(k0, j0, c); });
          fn = weno_value<true>(wrap(i0, nx), nx, uf, [&](int c) { return TN.at(k0, j0, c); });
        } else if (ax == 1) {
          const D uf = Vc.at(k0, j0, i0);
          f1 = weno_value<true>(wrap(j0, ny), ny, uf, [&](int c) { return T1.at(k0, c, i0); });
          fn = weno_value<true>(wrap(j0, ny), ny, uf, [&](int c) { return TN.at(k0, c, i0); });
        } else {
          const D uf = Wc.at(k0, j0, i0);
          f1 = weno_value<false>(k0, nz, uf, [&](int c) { return T1.at(c, j0, i0); });
          fn = weno_value<false>(k0, nz, uf, [&](int c) { return TN.at(c, j0, i0); });
        }
      }
      s += 0.5 * a.dt * f1 * (lam.p[m][p1] - lam.p[m][p0]) + a.dt * fn * (lt1.p[m][p1] - lt1.p[m][p0]);
    }
    return s;
  };
  // u face (between cells i and i+1)
  {
    auto cu = [&](int c) -> D {
      return (LL(3, k, j - 1, c) - LL(3, k, j + 1, c)) * h * a.ihy + (LL(6, k - 1, j, c) - LL(6, k + 1, j, c)) * h * a.ihz;
    };
    lu[id] = lu_in[id] + (LL(0, k, j, i) - LL(0, k, j, i + 1)) * a.ihx + h * (cu(i) + cu(i + 1)) +
             adv(i, j, k, i + 1, j, k, 0) * a.ihx;
  }
  // v face (between cells j and j+1)
  {
    auto cv = [&](int c) -> D {
      return (LL(1, k, c, i - 1) - LL(1, k, c, i + 1)) * h * a.ihx + (LL(7, k - 1, c, i) - LL(7, k + 1, c, i)) * h * a.ihz;
    };
    lv[id] = lv_in[id] + (LL(4, k, j, i) - LL(4, k, j + 1, i)) * a.ihy + h * (cv(j) + cv(j + 1)) +
             adv(i, j, k, i, j + 1, k, 1) * a.ihy;
  }
  // w face (between layers k and k+1); the top wall carries no unknown
  if (k < nz - 1) {
    auto cw = [&](int c) -> D {
      return (LL(2, c, j, i - 1) - LL(2, c, j, i + 1)) * h * a.ihx + (LL(5, c, j - 1, i) - LL(5, c, j + 1, i)) * h * a.ihy;
    };
    lw[id] = lw_in[id] + (LL(8, k, j, i) - LL(8, k + 1, j, i)) * a.ihz + h * (cw(k) + cw(k + 1)) +
             adv(i, j, k, i, j, k + 1, 2) * a.ihz;
  } else {
    lw[id] = 0.0;
  }
}

// ---- momentum: face-local factors ---------------------------------------------------------
// mu = (1/rho) lam_r; the adjoint of 1/rho at the face turned into the adjoint of the
// restricted phase field there (1/rho = 1 / mixture(phi)); the adjoint of G at the face from
// the capillary force; the Pe-partial of J = -c_j grad G (c_j = (rho1 - rho2) / (2 Pe)).
struct AdjMomOut {
  D* mu[3];
  D* lph[3];  // adjoint of phi restricted to the u, v, w faces (w: index k is the face k+1)
  D* lG[3];   // adjoint of G restricted to the faces
};

__global__ void __launch_bounds__(kBlock)
    k_adj_mom_faces(NsIn<D> in, Restricted<D> R, const D* __restrict__ lr, AdjMomOut o, int nx,
                    int ny, int nz, D ihx, D ihy, D ihz, StepConsts c, D* part) {
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  const int k = bz / 3;
  const int comp = bz - 3 * k;
  const int f = c.first;
  MomCtx<D> m{{in.un, in.unm1, nx, ny, nz, f, c.uwb[0], c.uwt[0]},
              {in.vn, in.vnm1, nx, ny, nz, f, c.uwb[1], c.uwt[1]},
              {in.wn, in.wnm1, nx, ny, nz, f},
              {in.pn, in.pnm1, nx, ny, nz, f},
              {in.pn, nullptr, nx, ny, nz, 1},
              {R.G_c, nx, ny, nz},
              {R.phi_c, nx, ny, nz},
              {R.mu_c, nx, ny, nz},
              {R.mu_xy, nx, ny, nz},
              {R.mu_xz, nx, ny},
              {R.mu_yz, nx, ny},
              {in.taun, in.taunm1, R.phi_c, nx, ny, nz, f},
              R,
              in.un, in.unm1, in.vn, in.vnm1, in.wn, in.wnm1,
              nx, ny, nz, f, in.viscoelastic,
              ihx, ihy, ihz,
              c.inv_dt, c.inv_re, c.inv_rho0, c.nu_m, c.k_sigma, c.c_j};
  const int nc = nx * ny * nz;
  const int id = (k * ny + j) * nx + i;
  D jgp = 0;
  if (comp == 2 && k == nz - 1) {
    o.mu[2][id] = 0;
    o.lph[2][id] = 0;
    o.lG[2][id] = 0;
  } else {
    MomTerms<D> t;
    D dphic;
    if (comp == 0) {
      t = mom_u(m, k, j, i, id);
      dphic = (m.phic.at(k, j, i + 1) - m.phic.at(k, j, i)) * ihx;
    } else if (comp == 1) {
      t = mom_v(m, k, j, i, id);
      dphic = (m.phic.at(k, j + 1, i) - m.phic.at(k, j, i)) * ihy;
    } else {
      t = mom_w(m, k, j, i, id);
      dphic = (m.phic.at(k + 1, j, i) - m.phic.at(k, j, i)) * ihz;
    }
    const D l = lr[comp * nc + id];
    const D mu = t.ri * l;
    const D lri = l * (t.jg + t.gps - c.inv_re * (t.pol + t.vis) - c.k_sigma * t.cap);
    o.mu[comp][id] = mu;
    o.lph[comp][id] = -lri * t.ri * t.ri * (0.5 * (c.rho1 - c.rho2));
    o.lG[comp][id] = -c.k_sigma * mu * dphic;
    jgp = -mu * t.jg / c.pe;
  }
  block_partial(jgp, part);
}

// ---- momentum: stress-like adjoints, diffusive flux, pressure levels ----------------------
struct StressOut {
  D *lX, *lY, *lZ, *lExy, *lExz, *lEyz;  // lExz, lEyz: nz + 1 layers (edge m at z = m hz)
  D *lph_xy, *lph_xz, *lph_yz;           // adjoint of phi restricted to the edges
  D *lj[3];                              // adjoint of J at centres
  D *J[3];                               // J at centres (forward value)
};

__global__ void __launch_bounds__(kBlock)
    k_adj_stress(NsIn<D> in, Restricted<D> R, const D* __restrict__ lr, AdjMomOut mo, StressOut o,
                 D* __restrict__ lp_n, D* __restrict__ lp_nm1, int nx, int ny, int nz, D ihx, D ihy,
                 D ihz, StepConsts c) {
  int k, j, i;
  cell_index(k, j, i);
  const int nc = nx * ny * nz;
  const int id = (k * ny + j) * nx + i;
  const int f = c.first;
  const D h = 0.5;
  // forward velocities with the no-slip ghosts of eq. NS13 (2 u_w - adjacent)
  const Field<D> U{in.un, in.unm1, nx, ny, nz, f, c.uwb[0], c.uwt[0]},
      V{in.vn, in.vnm1, nx, ny, nz, f, c.uwb[1], c.uwt[1]}, W{in.wn, in.wnm1, nx, ny, nz, f};
  auto at = [&](const D* a, int kk, int jj, int ii) -> D { return a[(kk * ny + wrap(jj, ny)) * nx + wrap(ii, nx)]; };
  // face values with the wall rules: w faces exist for k in [0, nz-2]
  auto muf = [&](int comp, int kk, int jj, int ii) -> D {
    if (kk < 0 || kk >= nz || (comp == 2 && kk >= nz - 1)) return 0.0;
    return at(mo.mu[comp], kk, jj, ii);
  };
  auto nu = [&](int comp, int kk, int jj, int ii) -> D { return -c.inv_re * muf(comp, kk, jj, ii); };
  // centres
  const D lX = (nu(0, k, j, i - 1) - nu(0, k, j, i)) * ihx;
  const D lY = (nu(1, k, j - 1, i) - nu(1, k, j, i)) * ihy;
  const D lZ = (nu(2, k - 1, j, i) - nu(2, k, j, i)) * ihz;
  o.lX[id] = lX;
  o.lY[id] = lY;
  o.lZ[id] = lZ;
  // xy edge (i, j) at ((i+1) hx, (j+1) hy)
  const D lExy = (nu(0, k, j, i) - nu(0, k, j + 1, i)) * ihy + (nu(1, k, j, i) - nu(1, k, j, i + 1)) * ihx;
  o.lExy[id] = lExy;
  const D dmu = 0.5 * (c.mu1 - c.mu2);
  o.lph_xy[id] = lExy * ((U.s(k, j + 1, i) - U.s(k, j, i)) * ihy + (V.s(k, j, i + 1) - V.s(k, j, i)) * ihx) * dmu;
  // xz / yz edges of layer m (z = m hz): this cell's top edge m = k + 1, and m = 0 for k = 0
  auto zedges = [&](int mm) {
    const int e = (mm * ny + j) * nx + i;
    const D exz = (nu(0, mm - 1, j, i) - nu(0, mm, j, i)) * ihz + (nu(2, mm - 1, j, i) - nu(2, mm - 1, j, i + 1)) * ihx;
    const D eyz = (nu(1, mm - 1, j, i) - nu(1, mm, j, i)) * ihz + (nu(2, mm - 1, j, i) - nu(2, mm - 1, j + 1, i)) * ihy;
    o.lExz[e] = exz;
    o.lEyz[e] = eyz;
    const D sxz = (U.sd(mm, j, i) - U.sd(mm - 1, j, i)) * ihz + (W.sw(mm - 1, j, i + 1) - W.sw(mm - 1, j, i)) * ihx;
    const D syz = (V.sd(mm, j, i) - V.sd(mm - 1, j, i)) * ihz + (W.sw(mm - 1, j + 1, i) - W.sw(mm - 1, j, i)) * ihy;
    o.lph_xz[e] = exz * sxz * dmu;
    o.lph_yz[e] = eyz * syz * dmu;
  };
  zedges(k + 1);
  if (k == 0) zedges(0);
  // adjoint of J at this centre: J enters every face through the two-point mean of its
  // neighbouring centres, multiplied by the centred velocity difference there
  {
    auto du = [&](int comp, int kk, int jj, int ii, int dir) -> D {
      const Field<D>& F = comp == 0 ? U : (comp == 1 ? V : W);
      if (comp == 2) {
        if (dir == 0) return (F.sw(kk, jj, ii + 1) - F.sw(kk, jj, ii - 1)) * h * ihx;
        if (dir == 1) return (F.sw(kk, jj + 1, ii) - F.sw(kk, jj - 1, ii)) * h * ihy;
        return (F.sw(kk + 1, jj, ii) - F.sw(kk - 1, jj, ii)) * h * ihz;
      }
      if (dir == 0) return (F.s(kk, jj, ii + 1) - F.s(kk, jj, ii - 1)) * h * ihx;
      if (dir == 1) return (F.s(kk, jj + 1, ii) - F.s(kk, jj - 1, ii)) * h * ihy;
      return (F.sd(kk + 1, jj, ii) - F.sd(kk - 1, jj, ii)) * h * ihz;
    };
    for (int dir = 0; dir < 3; ++dir) {
      D s = muf(0, k, j, i) * du(0, k, j, i, dir) + muf(0, k, j, i - 1) * du(0, k, j, i - 1, dir);
      s += muf(1, k, j, i) * du(1, k, j, i, dir) + muf(1, k, j - 1, i) * du(1, k, j - 1, i, dir);
      if (k < nz - 1) s += muf(2, k, j, i) * du(2, k, j, i, dir);
      if (k > 0) s += muf(2, k - 1, j, i) * du(2, k - 1, j, i, dir);
      o.lj[dir][id] = h * s;
    }
    // forward J at the centre, kept for the velocity adjoint
    const Coarse<D> Gc{R.G_c, nx, ny, nz};
    o.J[0][id] = -c.c_j * (Gc.at(k, j, i + 1) - Gc.at(k, j, i - 1)) * h * ihx;
    o.J[1][id] = -c.c_j * (Gc.at(k, j + 1, i) - Gc.at(k, j - 1, i)) * h * ihy;
    o.J[2][id] = -c.c_j * (Gc.atn(k + 1, j, i) - Gc.atn(k - 1, j, i)) * h * ihz;
  }
  // pressure levels: grad p^n / rho0 and (1/rho - 1/rho0) grad p* transposed (grad^T = -div)
  {
    auto lrf = [&](int comp, int kk, int jj, int ii) -> D {
      if (kk < 0 || (comp == 2 && kk >= nz - 1)) return 0.0;
      return lr[comp * nc + (kk * ny + wrap(jj, ny)) * nx + wrap(ii, nx)];
    };
    auto rif = [&](int comp, int kk, int jj, int ii) -> D {
      if (kk < 0 || (comp == 2 && kk >= nz - 1)) return 0.0;
      const D* r = comp == 0 ? R.ri_x : (comp == 1 ? R.ri_y : R.ri_z);
      return at(r, kk, jj, ii) - c.inv_rho0;
    };
    const D div_n = (lrf(0, k, j, i) - lrf(0, k, j, i - 1)) * ihx + (lrf(1, k, j, i) - lrf(1, k, j - 1, i)) * ihy +
                    (lrf(2, k, j, i) - lrf(2, k - 1, j, i)) * ihz;
    const D div_s = (rif(0, k, j, i) * lrf(0, k, j, i) - rif(0, k, j, i - 1) * lrf(0, k, j, i - 1)) * ihx +
                    (rif(1, k, j, i) * lrf(1, k, j, i) - rif(1, k, j - 1, i) * lrf(1, k, j - 1, i)) * ihy +
                    (rif(2, k, j, i) * lrf(2, k, j, i) - rif(2, k - 1, j, i) * lrf(2, k - 1, j, i)) * ihz;
    const D lpn = -div_n * c.inv_rho0;
    const D lps = -div_s;
    // lp_nm1 holds the adjoint of p^{n+1} on entry (p^{n+1} = p^n + p'); lp_n the adjoint of
    // the level p^n of the later state
    const D lpnew = lp_nm1[id];
    lp_n[id] += lpnew + lpn + (f ? lps : 2.0 * lps);
    lp_nm1[id] = f ? 0.0 : -lps;
  }
}

// ---- momentum: centred adjoints (polymer stress, phi at centres, G at centres) -------------
struct CentreOut {
  D* lph_c;  // adjoint of phi restricted to centres (through T, the capillary force, mu_c)
  D* lG_c;   // adjoint of G restricted to centres (through J)
};

__global__ void __launch_bounds__(kBlock)
    k_adj_centre(NsIn<D> in, Restricted<D> R, AdjMomOut mo, StressOut so, CentreOut o,
                 SixOut out_tau0, SixOut out_tau1, int nx, int ny, int nz, D ihx, D ihy, D ihz,
                 StepConsts c) {
  int k, j, i;
  cell_index(k, j, i);
  const int id = (k * ny + j) * nx + i;
  const int f = c.first;
  const D h = 0.5, q = 0.25;
  // forward velocities with the no-slip ghosts of eq. NS13 (2 u_w - adjacent)
  const Field<D> U{in.un, in.unm1, nx, ny, nz, f, c.uwb[0], c.uwt[0]},
      V{in.vn, in.vnm1, nx, ny, nz, f, c.uwb[1], c.uwt[1]}, W{in.wn, in.wnm1, nx, ny, nz, f};
  auto at = [&](const D* a, int kk, int jj, int ii) -> D { return a[(kk * ny + wrap(jj, ny)) * nx + wrap(ii, nx)]; };
  const D lX = so.lX[id], lY = so.lY[id], lZ = so.lZ[id];
  const D phic = R.phi_c[id];
  D lphic = 0;
  if (in.viscoelastic) {
    D lT[6];
    lT[0] = lX;
    lT[1] = lY;
    lT[2] = lZ;
    lT[3] = q * (at(so.lExy, k, j, i) + at(so.lExy, k, j, i - 1) + at(so.lExy, k, j - 1, i) + at(so.lExy, k, j - 1, i - 1));
    // z edges: the Neumann clamp at the walls makes the wall edges take the adjacent layer twice
    auto S4 = [&](int mm) { return at(so.lExz, mm, j, i) + at(so.lExz, mm, j, i - 1); };
    auto S5 = [&](int mm) { return at(so.lEyz, mm, j, i) + at(so.lEyz, mm, j - 1, i); };
    lT[4] = q * (S4(k) + S4(k + 1) + (k == 0 ? S4(0) : 0.0) + (k == nz - 1 ? S4(nz) : 0.0));
    lT[5] = q * (S5(k) + S5(k + 1) + (k == 0 ? S5(0) : 0.0) + (k == nz - 1 ? S5(nz) : 0.0));
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const Field<D> t{in.taun[m], in.taunm1[m], nx, ny, nz, f};
      const D ts = t.s(k, j, i);
      const D lts = h * (1.0 + phic) * lT[m];
      lphic += h * ts * lT[m];
      out_tau0.p[m][id] += f ? lts : 2.0 * lts;
      out_tau1.p[m][id] = f ? 0.0 : -lts;
    }
  }
  // solvent viscosity at the centre: normal viscous stresses 2 mu_c d_a u_a
  const D lmu_c = 2.0 * (lX * (U.s(k, j, i) - U.s(k, j, i - 1)) * ihx + lY * (V.s(k, j, i) - V.s(k, j - 1, i)) * ihy +
                         lZ * (W.sw(k, j, i) - W.sw(k - 1, j, i)) * ihz);
  // capillary force G_face (phi_c(+) - phi_c) / h transposed onto phi_c
  auto A = [&](int comp, int kk, int jj, int ii) -> D {
    if (kk < 0 || (comp == 2 && kk >= nz - 1)) return 0.0;
    const D* g = comp == 0 ? R.G_x : (comp == 1 ? R.G_y : R.G_z);
    return -c.k_sigma * at(mo.mu[comp], kk, jj, ii) * at(g, kk, jj, ii);
  };
  lphic += (A(0, k, j, i - 1) - A(0, k, j, i)) * ihx + (A(1, k, j - 1, i) - A(1, k, j, i)) * ihy +
           (A(2, k - 1, j, i) - A(2, k, j, i)) * ihz;
  o.lph_c[id] = lphic + lmu_c * 0.5 * (c.mu1 - c.mu2);
  // J = -c_j grad G (2h central differences, Neumann in z) transposed: odd ghosts in z
  auto ljz = [&](int kk) -> D {
    if (kk < 0) return -at(so.lj[2], 0, j, i);
    if (kk >= nz) return -at(so.lj[2], nz - 1, j, i);
    return at(so.lj[2], kk, j, i);
  };
  o.lG_c[id] = -c.c_j * ((at(so.lj[0], k, j, i - 1) - at(so.lj[0], k, j, i + 1)) * h * ihx +
                         (at(so.lj[1], k, j - 1, i) - at(so.lj[1], k, j + 1, i)) * h * ihy +
                         (ljz(k - 1) - ljz(k + 1)) * h * ihz);
}

// ---- momentum: velocity levels --------------------------------------------------------------
struct VelOut {
  D *u0, *u1, *v0, *v1, *w0, *w1;  // adjoint of the velocity levels n (accumulated), n-1 (set)
};

__global__ void __launch_bounds__(kBlock)
    k_adj_mom_vel(NsIn<D> in, Restricted<D> R, const D* __restrict__ lr, AdjMomOut mo, StressOut so,
                  VelOut o, int nx, int ny, int nz, D ihx, D ihy, D ihz, StepConsts c) {
  int k, j, i;
  cell_index(k, j, i);
  const int nc = nx * ny * nz;
  const int id = (k * ny + j) * nx + i;
  const int f = c.first;
  const D h = 0.5;
  // forward velocities with the no-slip ghosts of eq. NS13 (2 u_w - adjacent)
  const Field<D> U{in.un, in.unm1, nx, ny, nz, f, c.uwb[0], c.uwt[0]},
      V{in.vn, in.vnm1, nx, ny, nz, f, c.uwb[1], c.uwt[1]}, W{in.wn, in.wnm1, nx, ny, nz, f};
  auto at = [&](const D* a, int kk, int jj, int ii) -> D { return a[(kk * ny + wrap(jj, ny)) * nx + wrap(ii, nx)]; };
  // lam_r with the wall rules: u, v odd ghosts beyond the walls (for the Dirichlet Laplacian);
  // w faces k in [0, nz-2], zero elsewhere
  auto Lu = [&](int kk, int jj, int ii) -> D {
    if (kk < 0) return -at(lr, 0, jj, ii);
    if (kk >= nz) return -at(lr, nz - 1, jj, ii);
    return at(lr, kk, jj, ii);
  };
  auto Lv = [&](int kk, int jj, int ii) -> D {
    if (kk < 0) return -at(lr + nc, 0, jj, ii);
    if (kk >= nz) return -at(lr + nc, nz - 1, jj, ii);
    return at(lr + nc, kk, jj, ii);
  };
  auto Lw = [&](int kk, int jj, int ii) -> D {
    if (kk < 0 || kk >= nz - 1) return 0.0;
    return at(lr + 2 * nc, kk, jj, ii);
  };
  auto muf = [&](int comp, int kk, int jj, int ii) -> D {
    if (kk < 0 || kk >= nz || (comp == 2 && kk >= nz - 1)) return 0.0;
    return at(mo.mu[comp], kk, jj, ii);
  };
  auto Jc = [&](int d, int kk, int jj, int ii) -> D { return at(so.J[d], min(max(kk, 0), nz - 1), jj, ii); };
  const D ihx2 = ihx * ihx, ihy2 = ihy * ihy, ihz2 = ihz * ihz;
  // edge products of the advection: xy edge (ii, jj) in layer kk
  auto lPxy = [&](int kk, int jj, int ii) -> D {
    return (Lu(kk, jj, ii) - Lu(kk, jj + 1, ii)) * ihy + (Lv(kk, jj, ii) - Lv(kk, jj, ii + 1)) * ihx;
  };
  // xz edge between layers kk and kk+1 (kk in [0, nz-2]) at x face ii
  auto lPxz = [&](int kk, int jj, int ii) -> D {
    if (kk < 0 || kk >= nz - 1) return 0.0;
    return (Lu(kk, jj, ii) - Lu(kk + 1, jj, ii)) * ihz + (Lw(kk, jj, ii) - Lw(kk, jj, ii + 1)) * ihx;
  };
  auto lPyz = [&](int kk, int jj, int ii) -> D {
    if (kk < 0 || kk >= nz - 1) return 0.0;
    return (Lv(kk, jj, ii) - Lv(kk + 1, jj, ii)) * ihz + (Lw(kk, jj, ii) - Lw(kk, jj + 1, ii)) * ihy;
  };
  auto Mxy = [&](int kk, int jj, int ii) -> D { return at(R.mu_xy, kk, jj, ii) * at(so.lExy, kk, jj, ii); };
  auto Mxz = [&](int mm, int jj, int ii) -> D { return at(R.mu_xz, mm, jj, ii) * at(so.lExz, mm, jj, ii); };
  auto Myz = [&](int mm, int jj, int ii) -> D { return at(R.mu_yz, mm, jj, ii) * at(so.lEyz, mm, jj, ii); };
  auto lX = [&](int kk, int jj, int ii) -> D { return at(R.mu_c, kk, jj, ii) * at(so.lX, kk, jj, ii); };
  auto lY = [&](int kk, int jj, int ii) -> D { return at(R.mu_c, kk, jj, ii) * at(so.lY, kk, jj, ii); };
  auto lZ = [&](int kk, int jj, int ii) -> D { return at(R.mu_c, kk, jj, ii) * at(so.lZ, kk, jj, ii); };
  // ---- u face
  {
    D s = c.nu_m * ((Lu(k, j, i + 1) - 2 * Lu(k, j, i) + Lu(k, j, i - 1)) * ihx2 +
                    (Lu(k, j + 1, i) - 2 * Lu(k, j, i) + Lu(k, j - 1, i)) * ihy2 +
                    (Lu(k + 1, j, i) - 2 * Lu(k, j, i) + Lu(k - 1, j, i)) * ihz2);
    // advection: centre squares, xy and xz edge products
    auto Cc = [&](int ii) { return h * (U.s(k, j, ii - 1) + U.s(k, j, ii)); };
    auto lC = [&](int ii) { return (Lu(k, j, ii - 1) - Lu(k, j, ii)) * ihx; };
    s += lC(i) * Cc(i) + lC(i + 1) * Cc(i + 1);
    auto Ve = [&](int jj) { return h * (V.s(k, jj, i) + V.s(k, jj, i + 1)); };
    s += h * (lPxy(k, j, i) * Ve(j) + lPxy(k, j - 1, i) * Ve(j - 1));
    auto Wx = [&](int kk) { return h * (W.sw(kk, j, i) + W.sw(kk, j, i + 1)); };
    s += h * (lPxz(k, j, i) * Wx(k) + lPxz(k - 1, j, i) * Wx(k - 1));
    // J . grad u*
    auto Aux = [&](int ii) { return muf(0, k, j, ii) * h * (Jc(0, k, j, ii) + Jc(0, k, j, ii + 1)); };
    auto Auy = [&](int jj) { return muf(0, k, jj, i) * h * (Jc(1, k, jj, i) + Jc(1, k, jj, i + 1)); };
    auto Auz = [&](int kk) {
      kk = min(max(kk, 0), nz - 1);
      return muf(0, kk, j, i) * h * (Jc(2, kk, j, i) + Jc(2, kk, j, i + 1));
    };
    s += (Aux(i - 1) - Aux(i + 1)) * h * ihx + (Auy(j - 1) - Auy(j + 1)) * h * ihy + (Auz(k - 1) - Auz(k + 1)) * h * ihz;
    // viscous
    s += 2.0 * (lX(k, j, i) - lX(k, j, i + 1)) * ihx;
    s += (Mxy(k, j - 1, i) - Mxy(k, j, i)) * ihy;
    s += (Mxz(k, j, i) - Mxz(k + 1, j, i)) * ihz;
    if (k == 0) s += Mxz(0, j, i) * ihz;
    if (k == nz - 1) s -= Mxz(nz, j, i) * ihz;
    const D lh = -at(lr, k, j, i) * c.inv_dt;
    o.u0[id] += f ? s + lh : 2.0 * (s + lh);
    o.u1[id] = f ? 0.0 : -s - 0.5 * lh;
  }
  // ---- v face
  {
    D s = c.nu_m * ((Lv(k, j, i + 1) - 2 * Lv(k, j, i) + Lv(k, j, i - 1)) * ihx2 +
                    (Lv(k, j + 1, i) - 2 * Lv(k, j, i) + Lv(k, j - 1, i)) * ihy2 +
                    (Lv(k + 1, j, i) - 2 * Lv(k, j, i) + Lv(k - 1, j, i)) * ihz2);
    auto Cc = [&](int jj) { return h * (V.s(k, jj - 1, i) + V.s(k, jj, i)); };
    auto lC = [&](int jj) { return (Lv(k, jj - 1, i) - Lv(k, jj, i)) * ihy; };
    s += lC(j) * Cc(j) + lC(j + 1) * Cc(j + 1);
    auto Ue = [&](int ii) { return h * (U.s(k, j, ii) + U.s(k, j + 1, ii)); };
    s += h * (lPxy(k, j, i) * Ue(i) + lPxy(k, j, i - 1) * Ue(i - 1));
    auto Wy = [&](int kk) { return h * (W.sw(kk, j, i) + W.sw(kk, j + 1, i)); };
    s += h * (lPyz(k, j, i) * Wy(k) + lPyz(k - 1, j, i) * Wy(k - 1));
    auto Avx = [&](int ii) { return muf(1, k, j, ii) * h * (Jc(0, k, j, ii) + Jc(0, k, j + 1, ii)); };
    auto Avy = [&](int jj) { return muf(1, k, jj, i) * h * (Jc(1, k, jj, i) + Jc(1, k, jj + 1, i)); };
    auto Avz = [&](int kk) {
      kk = min(max(kk, 0), nz - 1);
      return muf(1, kk, j, i) * h * (Jc(2, kk, j, i) + Jc(2, kk, j + 1, i));
    };
    s += (Avx(i - 1) - Avx(i + 1)) * h * ihx + (Avy(j - 1) - Avy(j + 1)) * h * ihy + (Avz(k - 1) - Avz(k + 1)) * h * ihz;
    s += 2.0 * (lY(k, j, i) - lY(k, j + 1, i)) * ihy;
    s += (Mxy(k, j, i - 1) - Mxy(k, j, i)) * ihx;
    s += (Myz(k, j, i) - Myz(k + 1, j, i)) * ihz;
    if (k == 0) s += Myz(0, j, i) * ihz;
    if (k == nz - 1) s -= Myz(nz, j, i) * ihz;
    const D lh = -at(lr + nc, k, j, i) * c.inv_dt;
    o.v0[id] += f ? s + lh : 2.0 * (s + lh);
    o.v1[id] = f ? 0.0 : -s - 0.5 * lh;
  }
  // ---- w face (k <= nz-2); the top wall's adjoint is zero in both levels
  if (k < nz - 1) {
    D s = c.nu_m * ((Lw(k, j, i + 1) - 2 * Lw(k, j, i) + Lw(k, j, i - 1)) * ihx2 +
                    (Lw(k, j + 1, i) - 2 * Lw(k, j, i) + Lw(k, j - 1, i)) * ihy2 +
                    (Lw(k + 1, j, i) - 2 * Lw(k, j, i) + Lw(k - 1, j, i)) * ihz2);
    auto Cc = [&](int kk) { return h * (W.sw(kk - 1, j, i) + W.sw(kk, j, i)); };
    auto lC = [&](int kk) { return (Lw(kk - 1, j, i) - Lw(kk, j, i)) * ihz; };
    s += lC(k) * Cc(k) + lC(k + 1) * Cc(k + 1);
    auto Uz = [&](int ii) { return h * (U.s(k, j, ii) + U.s(k + 1, j, ii)); };
    s += h * (lPxz(k, j, i) * Uz(i) + lPxz(k, j, i - 1) * Uz(i - 1));
    auto Vz = [&](int jj) { return h * (V.s(k, jj, i) + V.s(k + 1, jj, i)); };
    s += h * (lPyz(k, j, i) * Vz(j) + lPyz(k, j - 1, i) * Vz(j - 1));
    auto Awx = [&](int ii) { return muf(2, k, j, ii) * h * (Jc(0, k, j, ii) + Jc(0, k + 1, j, ii)); };
    auto Awy = [&](int jj) { return muf(2, k, jj, i) * h * (Jc(1, k, jj, i) + Jc(1, k + 1, jj, i)); };
    auto Awz = [&](int kk) -> D {
      if (kk < 0 || kk >= nz - 1) return 0.0;
      return muf(2, kk, j, i) * h * (Jc(2, kk, j, i) + Jc(2, kk + 1, j, i));
    };
    s += (Awx(i - 1) - Awx(i + 1)) * h * ihx + (Awy(j - 1) - Awy(j + 1)) * h * ihy + (Awz(k - 1) - Awz(k + 1)) * h * ihz;
    s += 2.0 * (lZ(k, j, i) - lZ(k + 1, j, i)) * ihz;
    s += (Mxz(k + 1, j, i - 1) - Mxz(k + 1, j, i)) * ihx;
    s += (Myz(k + 1, j - 1, i) - Myz(k + 1, j, i)) * ihy;
    const D lh = -at(lr + 2 * nc, k, j, i) * c.inv_dt;
    o.w0[id] += f ? s + lh : 2.0 * (s + lh);
    o.w1[id] = f ? 0.0 : -s - 0.5 * lh;
  } else {
    o.w0[id] = 0.0;
    o.w1[id] = 0.0;
  }
}

// ---- restriction transposed, with the chemical potential -----------------------------------
// Every coarse location averaged the fine cells around it with weight 1/2 per refined axis;
// transposed, each fine cell collects those weights from the locations that contain it. The
// z faces and z edges on the walls averaged the wall-adjacent fine cell twice.
struct RestrictAdjIn {
  const D *lG_c, *lG_x, *lG_y, *lG_z;          // nc (lG_z: index k is the face k+1)
  const D *lph_c, *lph_x, *lph_y, *lph_z;      // nc
  const D *lph_xy;                             // nc (xy edges)
  const D *lph_xz, *lph_yz;                    // nz + 1 layers
};

__global__ void __launch_bounds__(kBlock)
    k_adj_restrict_ch(RestrictAdjIn a, const D* __restrict__ lphi_new_in, D* __restrict__ lG_out,
                      D* __restrict__ lphi_out, int fnx, int fny, int fnz, D fihx, D fihy, D fihz,
                      int cnx, int cny, int cnz, int ry, D cn2, D S, D dwall) {
  int K, J, I;
  cell_index(K, J, I);
  const int id = (K * fny + J) * fnx + I;
  auto cat = [&](const D* p, int kk, int jj, int ii) -> D { return p[(kk * cny + jj) * cnx + ii]; };
  const D wyc = ry == 2 ? 0.5 : 1.0;
  auto lGf = [&](int Kf, int Jf, int If) -> D {
    Kf = min(max(Kf, 0), fnz - 1);
    Jf = wrap(Jf, fny);
    If = wrap(If, fnx);
    const int ic = If >> 1, ixf = ((If - 1) >> 1) & (cnx - 1);
    const int jc = ry == 2 ? (Jf >> 1) : 0, jyf = ry == 2 ? (((Jf - 1) >> 1) & (cny - 1)) : 0;
    const int kc = Kf >> 1, mz = (Kf + 1) >> 1;
    D s = 0.5 * wyc * 0.5 * cat(a.lG_c, kc, jc, ic);
    s += 0.5 * wyc * 0.5 * cat(a.lG_x, kc, jc, ixf);
    s += 0.5 * (ry == 2 ? 0.5 : 1.0) * 0.5 * cat(a.lG_y, kc, jyf, ic);
    if (mz >= 1 && mz <= cnz - 1) s += 0.5 * wyc * 0.5 * cat(a.lG_z, mz - 1, jc, ic);
    return s;
  };
  const D g0 = lGf(K, J, I);
  // phase field
  const int ic = I >> 1, ixf = ((I - 1) >> 1) & (cnx - 1);
  const int jc = ry == 2 ? (J >> 1) : 0, jyf = ry == 2 ? (((J - 1) >> 1) & (cny - 1)) : 0;
  const int kc = K >> 1, mz = (K + 1) >> 1;
  const D wyf = ry == 2 ? 0.5 : 1.0;
  const D wzf = (K == 0 || K == fnz - 1) ? 1.0 : 0.5;
  D lp = lphi_new_in[id];
  lp += 0.5 * wyc * 0.5 * cat(a.lph_c, kc, jc, ic);
  lp += 0.5 * wyc * 0.5 * cat(a.lph_x, kc, jc, ixf);
  lp += 0.5 * wyf * 0.5 * cat(a.lph_y, kc, jyf, ic);
  if (mz >= 1 && mz <= cnz - 1) lp += 0.5 * wyc * 0.5 * cat(a.lph_z, mz - 1, jc, ic);
  lp += 0.5 * wyf * 0.5 * cat(a.lph_xy, kc, jyf, ixf);
  lp += wzf * wyc * 0.5 * cat(a.lph_xz, mz, jc, ixf);
  lp += wzf * wyf * 0.5 * cat(a.lph_yz, mz, jyf, ic);
  // G = -Cn^2 (L_N phi + b) + S (phi - phi*) + f(phi*): phi enters through -Cn^2 L_N + S; with
  // relaxed walls (eq. NS34) also through -Cn^2 dwall on the wall-adjacent layers
  const D lap = (lGf(K, J, I + 1) - 2 * g0 + lGf(K, J, I - 1)) * fihx * fihx +
                (lGf(K, J + 1, I) - 2 * g0 + lGf(K, J - 1, I)) * fihy * fihy +
                (lGf(K + 1, J, I) - 2 * g0 + lGf(K - 1, J, I)) * fihz * fihz;
  const D wallw = (D)((K == 0) + (K == fnz - 1));
  lG_out[id] = g0;
  lphi_out[id] = lp - cn2 * lap + S * g0 - cn2 * dwall * wallw * g0;
}

// ---- Cahn-Hilliard right-hand side, wetting data and advection transposed -----------------
struct ChAdjIn {
  const D *lQ, *lG, *phin, *phinm1, *phinew;
  Prolonged<D> pv;
};

template <bool WENO>
__global__ void __launch_bounds__(kBlock)
    k_adj_ch(ChAdjIn a, D* __restrict__ lphi_n, D* __restrict__ lphi_nm1, int fnx, int fny, int fnz,
             D fihx, D fihy, D fihz, StepConsts c, D sin_bot, D* part_theta, D* part_pe) {
  int K, J, I;
  cell_index(K, J, I);
  const int id = (K * fny + J) * fnx + I;
  const bool first = c.first != 0;
  const D h = 0.5;
  auto fidx = [&](int kk, int jj, int ii) { return (kk * fny + wrap(jj, fny)) * fnx + wrap(ii, fnx); };
  auto Q = [&](int kk, int jj, int ii) -> D { return a.lQ[fidx(min(max(kk, 0), fnz - 1), jj, ii)]; };
  auto ps = [&](int kk, int jj, int ii) -> D {
    const int p = fidx(min(max(kk, 0), fnz - 1), jj, ii);
    return first ? a.phin[p] : 2.0 * a.phin[p] - a.phinm1[p];
  };
  const D lq = a.lQ[id];
  const D zeta = (Q(K, J, I + 1) - 2 * lq + Q(K, J, I - 1)) * fihx * fihx +
                 (Q(K, J + 1, I) - 2 * lq + Q(K, J - 1, I)) * fihy * fihy +
                 (Q(K + 1, J, I) - 2 * lq + Q(K - 1, J, I)) * fihz * fihz;
  const D lg = a.lG[id];
  const D p0 = ps(K, J, I);
  const D pn = a.phinew[id];
  const D ph = first ? a.phin[id] : 2.0 * a.phin[id] - 0.5 * a.phinm1[id];
  D lphis = (-c.S + 3 * p0 * p0 - 1) * lg + ((3 * p0 * p0 - 1) * c.inv_cn2 - c.s_cn2) * zeta;
  // wetting data b = g cos(theta) (1 - phi*^2) / hz on the wall layers; it enters G
  // directly and Q - L_N b through the solve. With relaxed walls (eq. NS34) the wall data are
  // b_R = b + (kappa / hz) phi_hat / gamma0 there, entering the same two places.
  D th = 0, lbw = 0;
  if (K == 0) {
    const D lb = -c.cn2 * lg - zeta;
    lphis += lb * c.g_bot * fihz * (-2.0 * p0);
    th = lb * (-sin_bot / (sqrt(2.0) * c.cn)) * fihz * (1.0 - p0 * p0);
    lbw += lb;
  }
  if (K == fnz - 1) {
    const D lb = -c.cn2 * lg - zeta;
    lphis += lb * c.g_top * fihz * (-2.0 * p0);
    lbw += lb;
  }
  // advection div(u phi*) transposed: lam_A = -(Pe/Cn^2) lam_Q
  auto lA = [&](int kk, int jj, int ii) -> D { return -c.pe_cn2 * Q(kk, jj, ii); };
  auto lfx = [&](int ii) { return (lA(K, J, ii) - lA(K, J, ii + 1)) * fihx; };
  auto lfy = [&](int jj) { return (lA(K, jj, I) - lA(K, jj + 1, I)) * fihy; };
  auto lfz = [&](int kk) -> D {
    if (kk < 0 || kk >= fnz - 1) return 0.0;
    return (lA(kk, J, I) - lA(kk + 1, J, I)) * fihz;
  };
  const int Jm = wrap(J - 1, fny), Im = wrap(I - 1, fnx);
  const D ufp = a.pv.uf(K, J, I), ufm = a.pv.uf(K, J, Im);
  const D vfp = a.pv.vf(K, J, I), vfm = a.pv.vf(K, Jm, I);
  const D wfp = a.pv.wf(K, J, I), wfm = a.pv.wf(K - 1, J, I);
  D A;  // forward advection at this cell, for the Pe-derivative of Q
  if (!WENO) {
    lphis += h * (lfx(I) * ufp + lfx(I - 1) * ufm) + h * (lfy(J) * vfp + lfy(J - 1) * vfm) +
             h * (lfz(K) * wfp + lfz(K - 1) * wfm);
    A = (ufp * h * (p0 + ps(K, J, I + 1)) - ufm * h * (ps(K, J, I - 1) + p0)) * fihx +
        (vfp * h * (p0 + ps(K, J + 1, I)) - vfm * h * (ps(K, J - 1, I) + p0)) * fihy +
        (wfp * h * (p0 + ps(K + 1, J, I)) - wfm * h * (ps(K - 1, J, I) + p0)) * fihz;
  } else {
    // WENO-Z face values: every face whose upwind stencil holds this cell
    lphis += weno_adj_axis<true>(
        I, fnx, [&](int c) { return ps(K, J, c); }, [&](int f) { return a.pv.uf(K, J, f); },
        [&](int f) { return lfx(f); });
    lphis += weno_adj_axis<true>(
        J, fny, [&](int c) { return ps(K, c, I); }, [&](int f) { return a.pv.vf(K, f, I); },
        [&](int f) { return lfy(f); });
    lphis += weno_adj_axis<false>(
        K, fnz, [&](int c) { return ps(c, J, I); }, [&](int f) { return a.pv.wf(f, J, I); },
        [&](int f) { return lfz(f); });
    auto vx = [&](int c) { return ps(K, J, c); };
    auto vy = [&](int c) { return ps(K, c, I); };
    auto vz = [&](int c) { return ps(c, J, I); };
    const D fzp = K < fnz - 1 ? wfp * weno_value<false>(K, fnz, wfp, vz) : 0.0;
    const D fzm = K > 0 ? wfm * weno_value<false>(K - 1, fnz, wfm, vz) : 0.0;
    A = (ufp * weno_value<true>(I, fnx, ufp, vx) - ufm * weno_value<true>(Im, fnx, ufm, vx)) * fihx +
        (vfp * weno_value<true>(J, fny, vfp, vy) - vfm * weno_value<true>(Jm, fny, vfm, vy)) * fihy +
        (fzp - fzm) * fihz;
  }
  // dJ/dPe: Q carries Pe explicitly and through S (S ~ sqrt(Pe)); the solve operator
  // D = L^2 - (S/Cn^2) L + gamma0 Pe/(dt Cn^2) and G carry it through S. Grouped so that the
  // O(1/dt) parts cancel pointwise.
  const D pe_part = (lq * ((ph - c.gamma0 * pn) * c.inv_dt - A) +
                     (c.S / (2.0 * c.pe)) * (zeta + c.cn2 * lg) * (pn - p0)) * c.inv_cn2;
  const D lphih = c.pe_cn2 * c.inv_dt * lq + c.relax_kappa * c.inv_gamma0 * fihz * lbw;
  lphi_n[id] += first ? lphis + lphih : 2.0 * (lphis + lphih);
  lphi_nm1[id] = first ? 0.0 : -lphis - 0.5 * lphih;
  block_partial(th, part_theta);
  block_partial(pe_part, part_pe);
}

// ---- prolongation transposed (eq. dual1): fine face adjoints gathered onto coarse faces -----
template <bool WENO>
__global__ void __launch_bounds__(kBlock)
    k_adj_prolong(ChAdjIn a, VelOut o, int cnx, int cny, int cnz, int fnx, int fny, int fnz,
                  D fihx, D fihy, D fihz, int ry, StepConsts c) {
  int k, j, i;
  cell_index(k, j, i);
  const int id = (k * cny + j) * cnx + i;
  const bool first = c.first != 0;
  const D h = 0.5;
  auto fidx = [&](int kk, int jj, int ii) { return (kk * fny + wrap(jj, fny)) * fnx + wrap(ii, fnx); };
  auto lA = [&](int kk, int jj, int ii) -> D { return -c.pe_cn2 * a.lQ[fidx(kk, jj, ii)]; };
  auto ps = [&](int kk, int jj, int ii) -> D {
    const int p = fidx(min(max(kk, 0), fnz - 1), jj, ii);
    return first ? a.phin[p] : 2.0 * a.phin[p] - a.phinm1[p];
  };
  // adjoint of the fine face velocities: flux adjoint times the face value of phi* (the face
  // mean, or the WENO-Z value from the side the face velocity picks)
  auto Lx = [&](int K, int J, int I) {
    I = wrap(I, fnx);
    const D fv = WENO ? weno_value<true>(I, fnx, a.pv.uf(K, J, I), [&](int c) { return ps(K, J, c); })
                      : h * (ps(K, J, I) + ps(K, J, I + 1));
    return (lA(K, J, I) - lA(K, J, I + 1)) * fihx * fv;
  };
  auto Ly = [&](int K, int J, int I) {
    J = wrap(J, fny);
    const D fv = WENO ? weno_value<true>(J, fny, a.pv.vf(K, J, I), [&](int c) { return ps(K, c, I); })
                      : h * (ps(K, J, I) + ps(K, J + 1, I));
    return (lA(K, J, I) - lA(K, J + 1, I)) * fihy * fv;
  };
  auto Lz = [&](int K, int J, int I) -> D {
    if (K < 0 || K >= fnz - 1) return 0.0;
    const D fv = WENO ? weno_value<false>(K, fnz, a.pv.wf(K, J, I), [&](int c) { return ps(c, J, I); })
                      : h * (ps(K, J, I) + ps(K + 1, J, I));
    return (lA(K, J, I) - lA(K + 1, J, I)) * fihz * fv;
  };
  D su = 0, sv = 0, sw = 0;
  for (int dz = 0; dz < 2; ++dz) {
    const int K = 2 * k + dz;
    for (int dy = 0; dy < ry; ++dy) {
      const int J = ry * j + dy;
      su += Lx(K, J, 2 * i + 1) + h * Lx(K, J, 2 * i) + h * Lx(K, J, 2 * i + 2);
    }
    for (int dx = 0; dx < 2; ++dx) {
      const int I = 2 * i + dx;
      if (ry == 2)
        sv += Ly(K, 2 * j + 1, I) + h * Ly(K, 2 * j, I) + h * Ly(K, 2 * j + 2, I);
      else
        sv += Ly(K, 0, I);
    }
  }
  if (k < cnz - 1)
    for (int dx = 0; dx < 2; ++dx)
      for (int dy = 0; dy < ry; ++dy) {
        const int I = 2 * i + dx, J = ry * j + dy;
        sw += Lz(2 * k + 1, J, I) + h * Lz(2 * k, J, I) + h * Lz(2 * k + 2, J, I);
      }
  o.u0[id] += first ? su : 2.0 * su;
  o.v0[id] += first ? sv : 2.0 * sv;
  o.w0[id] += first ? sw : 2.0 * sw;
  if (!first) {
    o.u1[id] -= su;
    o.v1[id] -= sv;
    o.w1[id] -= sw;
  }
}

// ---- gradient partial sums, fixed order -----------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_adj_final(const D* __restrict__ part, int n_wi, int off_pe1, int n_pe1, int off_th, int n_f,
                int off_pe2, D* __restrict__ grad3) {
  __shared__ D sh[3][kBlock];
  const int t = threadIdx.x;
  D th = 0, pe = 0, wi = 0;
  for (int b = t; b < n_wi; b += blockDim.x) wi += part[b];
  for (int b = t; b < n_pe1; b += blockDim.x) pe += part[off_pe1 + b];
  for (int b = t; b < n_f; b += blockDim.x) {
    th += part[off_th + b];
    pe += part[off_pe2 + b];
  }
  sh[0][t] = th;
  sh[1][t] = pe;
  sh[2][t] = wi;
  __syncthreads();
  // pairwise tree in a fixed order (blockDim.x is a power of two)
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      sh[0][t] += sh[0][t + h];
      sh[1][t] += sh[1][t + h];
      sh[2][t] += sh[2][t + h];
    }
    __syncthreads();
  }
  if (t < 3) grad3[t] += sh[t][0];
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------

int adj_blocks(int nx, int ny, int nz_blocks) {
  const Launch3 L = launch3(nx, ny, nz_blocks);
  return (int)(L.grid.x * L.grid.y * L.grid.z);
}

hipError_t launch_adj_polymer(const Dims& c, const StepConsts& k, const double* u, const double* v,
                              const double* w, const double* const lam_tau[6],
                              const double* const tau_n[6], const double* const tau_1[6],
                              double* const lt1[6], double* const lL[9], double* const out_tau0[6],
                              const double* lu_in, const double* lv_in, const double* lw_in,
                              double* lu, double* lv, double* lw, double* part, hipStream_t st) {
  PolyArgs a{u, v, w, c.nx, c.ny, c.nz, c.ihx, c.ihy, c.ihz, k.dt, k.inv_wi, 1.0 - k.beta,
             k.giesekus == 0.0 ? 0.0 : k.giesekus / (1.0 - k.beta), walls_of<double>(k)};
  Six lam, tn, t1, l1;
  SixOut lo, ot;
  Nine nl;
  for (int m = 0; m < 6; ++m) {
    lam.p[m] = lam_tau[m];
    tn.p[m] = tau_n[m];
    t1.p[m] = tau_1[m];
    l1.p[m] = lt1[m];
    lo.p[m] = lt1[m];
    ot.p[m] = out_tau0[m];
  }
  for (int m = 0; m < 9; ++m) nl.p[m] = lL[m];
  const Launch3 L = launch3(c.nx, c.ny, c.nz);
  const int nb = adj_blocks(c.nx, c.ny, c.nz);
  const bool weno = k.advection == 1;
  hipLaunchKernelGGL(weno ? k_adj_polymer_s2<true> : k_adj_polymer_s2<false>, L.grid, L.block, 0, st, a, lam, t1,
                     lo, part);
  hipLaunchKernelGGL(weno ? k_adj_polymer_s1<true> : k_adj_polymer_s1<false>, L.grid, L.block, 0, st, a, lam, l1,
                     tn, t1, ot, nl, part + nb);
  hipLaunchKernelGGL(weno ? k_adj_polymer_vel<true> : k_adj_polymer_vel<false>, L.grid, L.block, 0, st, a, lu_in,
                     lv_in, lw_in, lam, l1, tn, t1, nl, lu, lv, lw);
  return hipGetLastError();
}

hipError_t launch_adj_momentum(const Dims& c, const StepConsts& k, NsIn<double> in, Restricted<double> R,
                               const double* lr, const AdjMomBufs& b, double* lp_n, double* lp_nm1,
                               double* const out_tau0[6], double* const out_tau1[6], double* u0,
                               double* u1, double* v0, double* v1, double* w0, double* w1,
                               double* part, hipStream_t st) {
  AdjMomOut mo;
  StressOut so;
  CentreOut co;
  for (int a = 0; a < 3; ++a) {
    mo.mu[a] = b.mu[a];
    mo.lph[a] = b.lph_f[a];
    mo.lG[a] = b.lG_f[a];
    so.lj[a] = b.lj[a];
    so.J[a] = b.J[a];
  }
  so.lX = b.lX;
  so.lY = b.lY;
  so.lZ = b.lZ;
  so.lExy = b.lExy;
  so.lExz = b.lExz;
  so.lEyz = b.lEyz;
  so.lph_xy = b.lph_xy;
  so.lph_xz = b.lph_xz;
  so.lph_yz = b.lph_yz;
  co.lph_c = b.lph_c;
  co.lG_c = b.lG_c;
  SixOut t0, t1;
  for (int m = 0; m < 6; ++m) {
    t0.p[m] = out_tau0[m];
    t1.p[m] = out_tau1[m];
  }
  VelOut vo{u0, u1, v0, v1, w0, w1};
  const Launch3 L3 = launch3(c.nx, c.ny, 3 * c.nz);
  hipLaunchKernelGGL(k_adj_mom_faces, L3.grid, L3.block, 0, st, in, R, lr, mo, c.nx, c.ny, c.nz, c.ihx, c.ihy,
                     c.ihz, k, part);
  const Launch3 L = launch3(c.nx, c.ny, c.nz);
  hipLaunchKernelGGL(k_adj_stress, L.grid, L.block, 0, st, in, R, lr, mo, so, lp_n, lp_nm1, c.nx, c.ny, c.nz,
                     c.ihx, c.ihy, c.ihz, k);
  hipLaunchKernelGGL(k_adj_centre, L.grid, L.block, 0, st, in, R, mo, so, co, t0, t1, c.nx, c.ny, c.nz, c.ihx,
                     c.ihy, c.ihz, k);
  hipLaunchKernelGGL(k_adj_mom_vel, L.grid, L.block, 0, st, in, R, lr, mo, so, vo, c.nx, c.ny, c.nz, c.ihx,
                     c.ihy, c.ihz, k);
  return hipGetLastError();
}

hipError_t launch_adj_restrict_ch(const Dims& f, const Dims& c, const StepConsts& k, const AdjMomBufs& b,
                                  const double* lphi_new_in, double* lG, double* lphi, hipStream_t st) {
  RestrictAdjIn a{b.lG_c, b.lG_f[0], b.lG_f[1], b.lG_f[2], b.lph_c, b.lph_f[0], b.lph_f[1], b.lph_f[2],
                  b.lph_xy, b.lph_xz, b.lph_yz};
  const Launch3 L = launch3(f.nx, f.ny, f.nz);
  hipLaunchKernelGGL(k_adj_restrict_ch, L.grid, L.block, 0, st, a, lphi_new_in, lG, lphi, f.nx, f.ny, f.nz,
                     f.ihx, f.ihy, f.ihz, c.nx, c.ny, c.nz, c.ny == 1 ? 1 : 2, k.cn2, k.S,
                     -k.relax_kappa * f.ihz);
  return hipGetLastError();
}

hipError_t launch_adj_ch(const Dims& f, const Dims& c, const StepConsts& k, const double* lQ,
                         const double* lG, const double* phin, const double* phinm1,
                         const double* phinew, const double* un, const double* unm1, const double* vn,
                         const double* vnm1, const double* wn, const double* wnm1, double sin_bot,
                         double* lphi_n, double* lphi_nm1, double* u0, double* u1, double* v0,
                         double* v1, double* w0, double* w1, double* part_theta, double* part_pe,
                         hipStream_t st) {
  const int ry = c.ny == 1 ? 1 : 2;
  ChAdjIn a{lQ, lG, phin, phinm1, phinew, {un, unm1, vn, vnm1, wn, wnm1, c.nx, c.ny, c.nz, ry, k.first}};
  const Launch3 L = launch3(f.nx, f.ny, f.nz);
  const bool weno = k.advection == 1;
  hipLaunchKernelGGL(weno ? k_adj_ch<true> : k_adj_ch<false>, L.grid, L.block, 0, st, a, lphi_n, lphi_nm1, f.nx,
                     f.ny, f.nz, f.ihx, f.ihy, f.ihz, k, sin_bot, part_theta, part_pe);
  VelOut vo{u0, u1, v0, v1, w0, w1};
  const Launch3 Lc = launch3(c.nx, c.ny, c.nz);
  hipLaunchKernelGGL(weno ? k_adj_prolong<true> : k_adj_prolong<false>, Lc.grid, Lc.block, 0, st, a, vo, c.nx,
                     c.ny, c.nz, f.nx, f.ny, f.nz, f.ihx, f.ihy, f.ihz, ry, k);
  return hipGetLastError();
}

hipError_t launch_adj_final(const double* part, int n_wi, int off_pe1, int n_pe1, int off_th, int n_f,
                            int off_pe2, double* grad3, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(kBlock), 0, st, part, n_wi, off_pe1, n_pe1, off_th, n_f,
                     off_pe2, grad3);
  return hipGetLastError();
}

}  // namespace drpf
