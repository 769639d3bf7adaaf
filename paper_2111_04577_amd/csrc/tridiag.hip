// Wall-normal pass of the constant-coefficient solver: after the x and y transforms every
// Fourier mode (kx, ky) leaves a tridiagonal system across the walls,
//   a x_{k-1} + b_k x_k + a x_{k+1} = d_k,   b_k = coeff * (lam_x + lam_y) - 2a - shift,
// whose end rows carry the wall rule (Neumann ghost = adjacent, no-slip ghost = -adjacent,
// or the z-face form with zero wall values). The systems are solved by parallel cyclic
// reduction (PCR) in LDS: a block holds a tile of TL consecutive modes, one thread per
// (row, mode); the rows of a z level are contiguous in memory, so the tile is loaded and
// stored with coalesced accesses. Each of the log2(n) PCR steps eliminates the couplings
// at distance s from every row at once; the reciprocal of every diagonal is kept beside it
// so that a step costs one reciprocal per row. Every operator here is symmetric, which the
// reduction preserves and uses (pcr_sym).
//
// Passes:
//   zpass_ch  -- the two Helmholtz operators of the Dong splitting (eqs. NS26-NS27),
//                (L - c_psi) then (L + alpha), applied together per mode through the
//                wall-normal DCT-II that diagonalises both (see k_zpass_ch).
//   zpass_ns  -- the velocity Helmholtz solves of eq. NS36, the divergence of the predicted
//                velocity, the pressure-increment Poisson solve of eq. NS37 in FP64 with the
//                (0,0) mode pinned and its mean removed, and the correction of eq. NS38
//                (all per mode, in spectral x/y space).
//   zpass_helmholtz -- one generic solve (the drpf_helmholtz_solve entry point).
#include "kernels.hpp"
#include "lds_fft.hpp"
#include "lds_fft16.hpp"

namespace drpf {

namespace {

constexpr int kZBlock = 1024;  // most threads per block of the Cahn-Hilliard wall-normal pass

// Reciprocal of a diagonal entry: the hardware estimate refined by Newton-Raphson steps
// (r <- r + r (1 - b r)), one for FP32 and two for FP64, each squaring the relative error of
// the estimate; the diagonals of the projection's systems are far from zero and overflow.
__device__ __forceinline__ float recip(float b) {
  const float r = __builtin_amdgcn_rcpf(b);
  return fmaf(r, fmaf(-b, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return fma(r, fma(-b, r, 1.0), r);
}

// PCR over several symmetric systems at once: NM matrices with NR right-hand sides,
// right-hand side r belonging to matrix (MAP >> r) & 1, so that one barrier pair per
// reduction step serves them all. A reduction step keeps a symmetric matrix symmetric (the
// coupling of row i to row i - s equals that of row i - s to row i), so a row takes from each
// neighbour only its reciprocal diagonal, its outer coupling and its right-hand sides:
//   b_i <- b_i - a_i^2 / b_{i-s} - c_i^2 / b_{i+s},  a_i <- -a_i a_{i-s} / b_{i-s},
//   c_i <- -c_i c_{i+s} / b_{i+s},  d_i <- d_i - a_i d_{i-s} / b_{i-s} - c_i d_{i+s} / b_{i+s}.
// On entry (a, b, c, d) hold the thread's row (a = 0 on the first row, c = 0 on the last); on
// exit d holds the solution. LDS: NM planes each of a, c and 1/b, then NR complex planes,
// each [row][line] of n * TL entries.
template <typename A, int NM, int NR, int MAP>
__device__ __forceinline__ void pcr_sym(unsigned char* base, int n, int TL, int row, int line,
                                        A (&a)[NM], A (&b)[NM], A (&c)[NM], cx<A> (&d)[NR]) {
  const int plane = n * TL;
  const int me = row * TL + line;
  A* La = reinterpret_cast<A*>(base);
  A* Lc = La + NM * plane;
  A* Lib = Lc + NM * plane;
  cx<A>* Ld = reinterpret_cast<cx<A>*>(Lib + NM * plane);
  A ib[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) ib[m] = recip(b[m]);
  for (int s = 1; s < n; s <<= 1) {
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      La[m * plane + me] = a[m];
      Lc[m * plane + me] = c[m];
      Lib[m * plane + me] = ib[m];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) Ld[r * plane + me] = d[r];
    __syncthreads();
    A al[NM], ga[NM], am[NM], cp[NM];
    cx<A> dm[NR], dp[NR];
#pragma unroll
    for (int m = 0; m < NM; ++m) al[m] = ga[m] = am[m] = cp[m] = (A)0;
#pragma unroll
    for (int r = 0; r < NR; ++r) dm[r] = dp[r] = mk<A>(0, 0);
    if (row - s >= 0) {
      const int q = me - s * TL;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        al[m] = -a[m] * Lib[m * plane + q];
        am[m] = La[m * plane + q];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) dm[r] = Ld[r * plane + q];
    }
    if (row + s < n) {
      const int q = me + s * TL;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        ga[m] = -c[m] * Lib[m * plane + q];
        cp[m] = Lc[m * plane + q];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) dp[r] = Ld[r * plane + q];
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      b[m] = b[m] + al[m] * a[m] + ga[m] * c[m];
      a[m] = al[m] * am[m];
      c[m] = ga[m] * cp[m];
      ib[m] = recip(b[m]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int m = (MAP >> r) & 1;
      d[r] = mk<A>(d[r].re + al[m] * dm[r].re + ga[m] * dp[r].re, d[r].im + al[m] * dm[r].im + ga[m] * dp[r].im);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) d[r] = ib[(MAP >> r) & 1] * d[r];
}

template <typename A, int NM, int NR>
size_t pcr_sym_bytes(int n, int TL) {
  return (size_t)n * TL * (3 * NM * sizeof(A) + NR * sizeof(cx<A>));
}

int tile_lines(int n) { return n >= 1024 ? 1 : 1024 / n; }

// Lines per block: the default tile, halved while the grid would have fewer than `target`
// blocks. Small blocks keep the barrier rounds of a wall-normal pass cheap and let several
// blocks interleave on a CU; 2D grids have only nx/2 + 1 lines.
int spread_lines(int tl, int lines, int target) {
  while (tl > 1 && (lines + tl - 1) / tl < target) tl >>= 1;
  return tl;
}

// ---- generic Helmholtz (drpf_helmholtz_solve) ---------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024)
    k_zpass_helmholtz(cx<T>* __restrict__ S, int P, int Ny, int Nz, const double* __restrict__ lamx,
                      const double* __restrict__ lamy, double ihz2, int bc, double coeff,
                      double shift, double scale) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TL = blockDim.x / Nz;
  const int line = threadIdx.x % TL;
  const int row = threadIdx.x / TL;
  const int lines = P * Ny;
  const int l = xcd_block() * TL + line;
  const bool valid = l < lines;
  const int lc = valid ? l : lines - 1;
  int ky, kx;
  spec_mode(lc, P, Ny, ky, kx);
  const size_t stride = (size_t)lines;
  const double a = coeff * ihz2;
  const double dxy = coeff * (lamx[kx] + lamy[ky]) - shift;
  const bool pinned = bc == 0 && shift == 0.0 && kx == 0 && ky == 0;
  const int n = bc == 2 ? Nz - 1 : Nz;
  double ar = row == 0 ? 0.0 : a, cr = row == Nz - 1 ? 0.0 : a, br = dxy - 2 * a;
  if (bc == 0) {
    if (row == 0 || row == Nz - 1) br = dxy - a;
  } else if (bc == 1) {
    if (row == 0 || row == Nz - 1) br = dxy - 3 * a;
  } else {
    if (row == Nz - 2) cr = 0.0;
    if (row == Nz - 1) { ar = 0.0; br = 1.0; }
  }
  cx<double> d[1];
  d[0] = valid ? widen<double>(S[row * stride + l]) : mk<double>(0, 0);
  d[0] = scale * d[0];
  if (bc == 2 && row == Nz - 1) d[0] = mk<double>(0, 0);
  // the singular (0,0) Neumann line: the pseudo-inverse drops the z-mean of the right-hand
  // side first (the pinned row then reproduces the remaining equations exactly); every
  // thread takes part in the barriers
  {
    cx<double>* Ls = reinterpret_cast<cx<double>*>(smem);
    Ls[row * TL + line] = d[0];
    __syncthreads();
    if (pinned) {
      double mre = 0, mim = 0;
      for (int k = 0; k < Nz; ++k) {
        mre += Ls[k * TL + line].re;
        mim += Ls[k * TL + line].im;
      }
      d[0] = mk<double>(d[0].re - mre / Nz, d[0].im - mim / Nz);
    }
    __syncthreads();
  }
  if (pinned) {
    if (row == 0) { ar = 0.0; cr = 0.0; br = 1.0; d[0] = mk<double>(0, 0); }
    if (row == 1) ar = 0.0;
  }
  (void)n;
  {
    double a1[1] = {ar}, b1[1] = {br}, c1[1] = {cr};
    pcr_sym<double, 1, 1, 0>(smem, Nz, TL, row, line, a1, b1, c1, d);
  }
  // zero-mean of the pinned mode: every thread takes part in the barrier
  cx<double>* Ld = reinterpret_cast<cx<double>*>(smem);
  Ld[row * TL + line] = d[0];
  __syncthreads();
  if (pinned) {
    double mre = 0, mim = 0;
    for (int k = 0; k < Nz; ++k) {
      mre += Ld[k * TL + line].re;
      mim += Ld[k * TL + line].im;
    }
    d[0] = mk<double>(d[0].re - mre / Nz, d[0].im - mim / Nz);
  }
  if (valid) S[row * stride + l] = mk<T>((T)d[0].re, (T)d[0].im);
}

// ---- wall data of the generic solve moved to the right-hand side ----------------------
template <typename T>
__global__ void __launch_bounds__(256)
    k_wall_rhs(const T* __restrict__ rhs, const T* __restrict__ wall, T* __restrict__ out, int layer,
               int nz, int bc, T cb, T ct) {
  const size_t n = (size_t)layer * nz;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(id / layer);
    const size_t e = id - (size_t)k * layer;
    T r = rhs[id];
    if (bc == 2) {
      if (k == nz - 1) r = (T)0;
      if (k == 0) r -= cb * wall[e];
      if (k == nz - 2) r -= ct * wall[layer + e];
    } else {
      if (k == 0) r -= cb * wall[e];
      if (k == nz - 1) r -= ct * wall[layer + e];
    }
    out[id] = r;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_top_layer(const T* __restrict__ top, T* __restrict__ x, int layer, size_t base) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < layer; e += gridDim.x * blockDim.x) x[base + e] = top[e];
}

// ---- Cahn-Hilliard pair -------------------------------------------------------------
// Both CH operators have zero-flux walls, so the DCT-II across the walls diagonalises them
// exactly (eigenvalue lam_z(m) of the second difference for cos(pi m (k + 1/2) / nz)). The
// pair (L_N - c_psi)^-1 (L_N + alpha)^-1 becomes: forward DCT, one multiplication by the
// reciprocal of (lam - c_psi)(lam + alpha) per coefficient (recip: both factors are bounded
// away from zero, since lam <= 0, alpha < 0 < c_psi), inverse DCT. Each DCT is one length-nz complex
// FFT in LDS (Makhoul's even/odd reordering with a quarter-wave twiddle); the data are
// complex (x/y spectral coefficients), so the real and imaginary sequences are separated
// from the pair (V_m, V_{nz-m}). A block holds TL consecutive modes, each a line of the
// compile-time FFT form (lds_fft16.hpp), which serves FP32; k_zpass_ch_rt below is the same
// pass with the run-time form (lds_fft.hpp, columns in LDS), which serves FP64.
template <typename T, bool ROBIN, int LOGNZ>
__global__ void __launch_bounds__(kZBlock)
    k_zpass_ch(cx<T>* __restrict__ S, int P, int Ny, int TL,
               const double* __restrict__ lamx, const double* __restrict__ lamy,
               const double* __restrict__ lamz, const cx<T>* __restrict__ twz,
               const cx<T>* __restrict__ twq, double c_psi, double alpha, double scale, double dwall) {
  using F = FftPlan<LOGNZ, fft_lp<T>()>;
  constexpr int Nz = F::M;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);  // mode t at t LS, position n at pad(n)
  cx<T>* stw = buf + TL * F::LS;                 // twiddles of the length-Nz transform
  for (int e = threadIdx.x; e < Nz; e += blockDim.x) stw[e] = twz[e];
  const int lines = P * Ny;
  const int l0 = xcd_block() * TL;
  const size_t stride = (size_t)lines;
  const int ltl = __ffs(TL) - 1;  // TL is a power of two
  auto at = [&](int n, int t) -> cx<T>& { return buf[t * F::LS + F::pad(n)]; };
  for (int e = threadIdx.x; e < Nz * TL; e += blockDim.x) {
    const int row = e >> ltl, t = e & (TL - 1);
    const int l = l0 + t;
    const int pos = (row & 1) ? (Nz - 1 - (row >> 1)) : (row >> 1);
    at(pos, t) = l < lines ? S[row * stride + l] : mk<T>(0, 0);
  }
  __syncthreads();
  const int fb = threadIdx.x >> F::LT, fq = threadIdx.x & (F::T - 1);
  fft16<T, false, LOGNZ, fft_lp<T>()>(buf + fb * F::LS, fq, fb < TL, stw);
  const int half = Nz >> 1;
  const T hf = (T)0.5;
  const T cp = (T)c_psi, al = (T)alpha, sc = (T)scale;
  // forward DCT-II coefficient from (V_m, V_{N-m}): X = Re(w A) + i Re(w B),
  // A = (V_m + conj V_{N-m}) / 2, B = (V_m - conj V_{N-m}) / (2i)
  auto dct_out = [&](cx<T> V, cx<T> Vp, cx<T> w) -> cx<T> {
    const cx<T> A = hf * (V + conj(Vp));
    const cx<T> B = hf * mul_mi(V - conj(Vp));
    return mk<T>((w * A).re, (w * B).re);
  };
  // inverse: Y_m = conj(w_m) [(P_m + Q_{N-m}) + i (Q_m - P_{N-m})], X_N = 0
  auto inverse_in = [&](int m, int mr, int t, cx<T> Fm, cx<T> Fr) {
    if (mr != m) {
      at(m, t) = conj(twq[m]) * mk<T>(Fm.re + Fr.im, Fm.im - Fr.re);
      at(mr, t) = conj(twq[mr]) * mk<T>(Fr.re + Fm.im, Fr.im - Fm.re);
    } else if (m == 0) {
      at(0, t) = Fm;
    } else {
      at(m, t) = conj(twq[m]) * mk<T>(Fm.re + Fm.im, Fm.im - Fm.re);
    }
  };
  if (!ROBIN) {
    for (int e = threadIdx.x; e < (half + 1) * TL; e += blockDim.x) {
      const int m = e >> ltl, t = e & (TL - 1);
      const int l = min(l0 + t, lines - 1);
      int ky, kx;
      spec_mode(l, P, Ny, ky, kx);
      // the eigenvalue factors in the storage type: lambda <= 0, alpha < 0 < c_psi, so neither
      // factor cancels
      const T lxy = (T)(lamx[kx] + lamy[ky]);
      const int mr = (Nz - m) & (Nz - 1);  // partner N - m (0 and N/2 pair with themselves)
      const cx<T> Vm = at(m, t), Vr = at(mr, t);
      const T lm = lxy + (T)lamz[m];
      const cx<T> Fm = (sc * recip((lm - cp) * (lm + al))) * dct_out(Vm, Vr, twq[m]);
      cx<T> Fr = Fm;
      if (mr != m) {
        const T lr = lxy + (T)lamz[mr];
        Fr = (sc * recip((lr - cp) * (lr + al))) * dct_out(Vr, Vm, twq[mr]);
      }
      inverse_in(m, mr, t, Fm, Fr);
    }
  } else {
    // Relaxed walls (eq. NS34 with D_w > 0): the operator is (L - c_psi)(L + alpha) + L dW,
    // d = dwall on the two wall-adjacent rows, a rank-two change of the Neumann product that
    // the DCT diagonalises. With F0 = X / A (A = (lambda - c_psi)(lambda + alpha), X the DCT
    // of the right-hand side, both scaled) the solution is F_m = F0_m - G_m s_m, G_m = d
    // lambda_m c_m / (N A_m), c_m = cos(pi m / 2N) = (row 0 of the DCT basis), s_m the sum
    // (m even) or difference (m odd) of the two wall values; since the inverse transform is
    // x_k = sum_m W_m F_m cos(pi m (k + 1/2) / N), W = (1, 2, 2, ...), the sum and difference
    // solve sigma = P_e / (1 + H_e), delta = P_o / (1 + H_o) with P = 2 sum W c F0 and
    // H = 2 sum W c G over even or odd m. H >= 0 (d < 0, lambda <= 0, A > 0).
    // after the twiddles, rounded up to 16 bytes: the wall sums [TL][2], the partials
    // [NC][TL][6], then G [Nz][TL] in the storage type
    const int NC = min((int)(blockDim.x >> ltl), 16);
    const size_t so = ((size_t)(TL * F::LS + Nz) * sizeof(cx<T>) + 15) & ~(size_t)15;
    cx<double>* sd = reinterpret_cast<cx<double>*>(smem + so);
    double* part = reinterpret_cast<double*>(sd + 2 * TL);
    T* sG = reinterpret_cast<T*>(part + 6 * NC * TL);
    for (int e = threadIdx.x; e < (half + 1) * TL; e += blockDim.x) {
      const int m = e >> ltl, t = e & (TL - 1);
      const int l = min(l0 + t, lines - 1);
      int ky, kx;
      spec_mode(l, P, Ny, ky, kx);
      const T lxy = (T)(lamx[kx] + lamy[ky]);
      const int mr = (Nz - m) & (Nz - 1);
      const cx<T> Vm = at(m, t), Vr = at(mr, t);
      // 1/A once per entry: F0 = scale X / A and G = d lambda c / (N A)
      const T lm = lxy + (T)lamz[m];
      const T im = recip((lm - cp) * (lm + al));
      at(m, t) = (sc * im) * dct_out(Vm, Vr, twq[m]);
      sG[m * TL + t] = (T)dwall * lm * twq[m].re * im / (T)Nz;
      if (mr != m) {
        const T lr = lxy + (T)lamz[mr];
        const T ir = recip((lr - cp) * (lr + al));
        at(mr, t) = (sc * ir) * dct_out(Vr, Vm, twq[mr]);
        sG[mr * TL + t] = (T)dwall * lr * twq[mr].re * ir / (T)Nz;
      }
    }
    __syncthreads();
    // partial sums over m = ch, ch + NC, ... per mode, then their totals
    for (int e = threadIdx.x; e < NC * TL; e += blockDim.x) {
      const int t = e & (TL - 1), ch = e >> ltl;
      double acc[6] = {0, 0, 0, 0, 0, 0};  // P_e (re, im), P_o (re, im), H_e, H_o
      for (int m = ch; m < Nz; m += NC) {
        const double wc = (m == 0 ? 2.0 : 4.0) * (double)twq[m].re;
        const cx<T> Fv = at(m, t);
        const int o = (m & 1) * 2;
        acc[o] += wc * (double)Fv.re;
        acc[o + 1] += wc * (double)Fv.im;
        acc[4 + (m & 1)] += wc * (double)sG[m * TL + t];
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) part[(ch * TL + t) * 6 + q] = acc[q];
    }
    __syncthreads();
    // totals: one thread per (quantity, mode), into the first chunk's slots
    for (int e = threadIdx.x; e < 6 * TL; e += blockDim.x) {
      const int t = e % TL, q = e / TL;
      double a = 0;
      for (int ch = 0; ch < NC; ++ch) a += part[(ch * TL + t) * 6 + q];
      part[t * 6 + q] = a;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TL; t += blockDim.x) {
      const double* a = part + t * 6;
      sd[2 * t] = mk<double>(a[0] / (1.0 + a[4]), a[1] / (1.0 + a[4]));      // sigma
      sd[2 * t + 1] = mk<double>(a[2] / (1.0 + a[5]), a[3] / (1.0 + a[5]));  // delta
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (half + 1) * TL; e += blockDim.x) {
      const int m = e >> ltl, t = e & (TL - 1);
      const int mr = (Nz - m) & (Nz - 1);
      auto corrected = [&](int mm) -> cx<T> {
        const cx<T> Fv = at(mm, t);
        const cx<double> s = sd[2 * t + (mm & 1)];
        const double g = (double)sG[mm * TL + t];
        return mk<T>((T)((double)Fv.re - g * s.re), (T)((double)Fv.im - g * s.im));
      };
      const cx<T> Fm = corrected(m);
      const cx<T> Fr = mr != m ? corrected(mr) : Fm;
      inverse_in(m, mr, t, Fm, Fr);
    }
  }
  __syncthreads();
  fft16<T, true, LOGNZ, fft_lp<T>()>(buf + fb * F::LS, fq, fb < TL, stw);
  for (int e = threadIdx.x; e < Nz * TL; e += blockDim.x) {
    const int row = e >> ltl, t = e & (TL - 1);
    const int l = l0 + t;
    const int pos = (row & 1) ? (Nz - 1 - (row >> 1)) : (row >> 1);
    if (l < lines) S[row * stride + l] = at(pos, t);
  }
}

// The same pass with the transform length at run time (lds_fft): the FP64 form. TRANS (relaxed
// walls only) solves with the transposed operator, for the discrete adjoint.
template <typename T, bool ROBIN, bool TRANS = false>
__global__ void __launch_bounds__(1024)
    k_zpass_ch_rt(cx<T>* __restrict__ S, int P, int Ny, int Nz, int logNz, int TL,
               const double* __restrict__ lamx, const double* __restrict__ lamy,
               const double* __restrict__ lamz, const cx<T>* __restrict__ twz,
               const cx<T>* __restrict__ twq, double c_psi, double alpha, double scale, double dwall) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);  // [position][mode]
  cx<T>* stw = buf + Nz * TL;                    // twiddles of the length-Nz transform
  for (int e = threadIdx.x; e < Nz; e += blockDim.x) stw[e] = twz[e];
  const int lines = P * Ny;
  const int l0 = xcd_block() * TL;
  const size_t stride = (size_t)lines;
  const int ltl = __ffs(TL) - 1;  // TL is a power of two
  for (int e = threadIdx.x; e < Nz * TL; e += blockDim.x) {
    const int row = e >> ltl, t = e & (TL - 1);
    const int l = l0 + t;
    const int pos = (row & 1) ? (Nz - 1 - (row >> 1)) : (row >> 1);
    buf[(pos << ltl) + t] = l < lines ? S[row * stride + l] : mk<T>(0, 0);
  }
  __syncthreads();
  lds_fft<T, false, true>(buf, Nz, logNz, TL, ltl, stw);
  const int half = Nz >> 1;
  const T hf = (T)0.5;
  const T cp = (T)c_psi, al = (T)alpha, sc = (T)scale;
  // forward DCT-II coefficient from (V_m, V_{N-m}): X = Re(w A) + i Re(w B),
  // A = (V_m + conj V_{N-m}) / 2, B = (V_m - conj V_{N-m}) / (2i)
  auto dct_out = [&](cx<T> V, cx<T> Vp, cx<T> w) -> cx<T> {
    const cx<T> A = hf * (V + conj(Vp));
    const cx<T> B = hf * mul_mi(V - conj(Vp));
    return mk<T>((w * A).re, (w * B).re);
  };
  // inverse: Y_m = conj(w_m) [(P_m + Q_{N-m}) + i (Q_m - P_{N-m})], X_N = 0
  auto inverse_in = [&](int m, int mr, int t, cx<T> Fm, cx<T> Fr) {
    if (mr != m) {
      buf[m * TL + t] = conj(twq[m]) * mk<T>(Fm.re + Fr.im, Fm.im - Fr.re);
      buf[mr * TL + t] = conj(twq[mr]) * mk<T>(Fr.re + Fm.im, Fr.im - Fm.re);
    } else if (m == 0) {
      buf[t] = Fm;
    } else {
      buf[m * TL + t] = conj(twq[m]) * mk<T>(Fm.re + Fm.im, Fm.im - Fm.re);
    }
  };
  if (!ROBIN) {
    for (int e = threadIdx.x; e < (half + 1) * TL; e += blockDim.x) {
      const int m = e >> ltl, t = e & (TL - 1);
      const int l = min(l0 + t, lines - 1);
      int ky, kx;
      spec_mode(l, P, Ny, ky, kx);
      // the eigenvalue factors in the storage type: lambda <= 0, alpha < 0 < c_psi, so neither
      // factor cancels
      const T lxy = (T)(lamx[kx] + lamy[ky]);
      const int mr = (Nz - m) & (Nz - 1);  // partner N - m (0 and N/2 pair with themselves)
      const cx<T> Vm = buf[m * TL + t], Vr = buf[mr * TL + t];
      const T lm = lxy + (T)lamz[m];
      const cx<T> Fm = (sc * recip((lm - cp) * (lm + al))) * dct_out(Vm, Vr, twq[m]);
      cx<T> Fr = Fm;
      if (mr != m) {
        const T lr = lxy + (T)lamz[mr];
        Fr = (sc * recip((lr - cp) * (lr + al))) * dct_out(Vr, Vm, twq[mr]);
      }
      inverse_in(m, mr, t, Fm, Fr);
    }
  } else {
    // Relaxed walls (eq. NS34 with D_w > 0): the operator is (L - c_psi)(L + alpha) + L dW,
    // d = dwall on the two wall-adjacent rows, a rank-two change of the Neumann product that
    // the DCT diagonalises. With F0 = X / A (A = (lambda - c_psi)(lambda + alpha), X the DCT
    // of the right-hand side, both scaled) the solution is F_m = F0_m - G_m s_m, G_m = d
    // lambda_m c_m / (N A_m), c_m = cos(pi m / 2N) = (row 0 of the DCT basis), s_m the sum
    // (m even) or difference (m odd) of the two wall values; since the inverse transform is
    // x_k = sum_m W_m F_m cos(pi m (k + 1/2) / N), W = (1, 2, 2, ...), the sum and difference
    // solve sigma = P_e / (1 + H_e), delta = P_o / (1 + H_o) with P = 2 sum W c F0 and
    // H = 2 sum W c G over even or odd m. H >= 0 (d < 0, lambda <= 0, A > 0).
    // Transposed (TRANS): the operator is (L - c_psi)(L + alpha) + dW L, whose rank-two part
    // takes the wall values of L x instead of x: G_m = d c_m / (N A_m), and P and H weight each
    // term by lambda_m (P = 2 sum W lambda c F0, H = 2 sum W lambda c G, the same H as above).
    // after the twiddles, rounded up to 16 bytes: the wall sums [TL][2], the partials
    // [NC][TL][6], then G [Nz][TL] in the storage type
    const int NC = min((int)(blockDim.x >> ltl), 16);
    const size_t so = ((size_t)(Nz * TL + Nz) * sizeof(cx<T>) + 15) & ~(size_t)15;
    cx<double>* sd = reinterpret_cast<cx<double>*>(smem + so);
    double* part = reinterpret_cast<double*>(sd + 2 * TL);
    T* sG = reinterpret_cast<T*>(part + 6 * NC * TL);
    for (int e = threadIdx.x; e < (half + 1) * TL; e += blockDim.x) {
      const int m = e >> ltl, t = e & (TL - 1);
      const int l = min(l0 + t, lines - 1);
      int ky, kx;
      spec_mode(l, P, Ny, ky, kx);
      const T lxy = (T)(lamx[kx] + lamy[ky]);
      const int mr = (Nz - m) & (Nz - 1);
      const cx<T> Vm = buf[m * TL + t], Vr = buf[mr * TL + t];
      // 1/A once per entry: F0 = scale X / A and G = d lambda c / (N A)
      const T lm = lxy + (T)lamz[m];
      const T im = recip((lm - cp) * (lm + al));
      buf[m * TL + t] = (sc * im) * dct_out(Vm, Vr, twq[m]);
      sG[m * TL + t] = (T)dwall * (TRANS ? (T)1 : lm) * twq[m].re * im / (T)Nz;
      if (mr != m) {
        const T lr = lxy + (T)lamz[mr];
        const T ir = recip((lr - cp) * (lr + al));
        buf[mr * TL + t] = (sc * ir) * dct_out(Vr, Vm, twq[mr]);
        sG[mr * TL + t] = (T)dwall * (TRANS ? (T)1 : lr) * twq[mr].re * ir / (T)Nz;
      }
    }
    __syncthreads();
    // partial sums over m = ch, ch + NC, ... per mode, then their totals
    for (int e = threadIdx.x; e < NC * TL; e += blockDim.x) {
      const int t = e & (TL - 1), ch = e >> ltl;
      T lxy = (T)0;
      if (TRANS) {
        int ky, kx;
        spec_mode(min(l0 + t, lines - 1), P, Ny, ky, kx);
        lxy = (T)(lamx[kx] + lamy[ky]);
      }
      double acc[6] = {0, 0, 0, 0, 0, 0};  // P_e (re, im), P_o (re, im), H_e, H_o
      for (int m = ch; m < Nz; m += NC) {
        const double wc = (m == 0 ? 2.0 : 4.0) * (double)twq[m].re * (TRANS ? (double)(lxy + (T)lamz[m]) : 1.0);
        const cx<T> F = buf[m * TL + t];
        const int o = (m & 1) * 2;
        acc[o] += wc * (double)F.re;
        acc[o + 1] += wc * (double)F.im;
        acc[4 + (m & 1)] += wc * (double)sG[m * TL + t];
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) part[(ch * TL + t) * 6 + q] = acc[q];
    }
    __syncthreads();
    // totals: one thread per (quantity, mode), into the first chunk's slots
    for (int e = threadIdx.x; e < 6 * TL; e += blockDim.x) {
      const int t = e % TL, q = e / TL;
      double a = 0;
      for (int ch = 0; ch < NC; ++ch) a += part[(ch * TL + t) * 6 + q];
      part[t * 6 + q] = a;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TL; t += blockDim.x) {
      const double* a = part + t * 6;
      sd[2 * t] = mk<double>(a[0] / (1.0 + a[4]), a[1] / (1.0 + a[4]));      // sigma
      sd[2 * t + 1] = mk<double>(a[2] / (1.0 + a[5]), a[3] / (1.0 + a[5]));  // delta
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (half + 1) * TL; e += blockDim.x) {
      const int m = e >> ltl, t = e & (TL - 1);
      const int mr = (Nz - m) & (Nz - 1);
      auto corrected = [&](int mm) -> cx<T> {
        const cx<T> F = buf[mm * TL + t];
        const cx<double> s = sd[2 * t + (mm & 1)];
        const double g = (double)sG[mm * TL + t];
        return mk<T>((T)((double)F.re - g * s.re), (T)((double)F.im - g * s.im));
      };
      const cx<T> Fm = corrected(m);
      const cx<T> Fr = mr != m ? corrected(mr) : Fm;
      inverse_in(m, mr, t, Fm, Fr);
    }
  }
  __syncthreads();
  lds_fft<T, true, true>(buf, Nz, logNz, TL, ltl, stw);
  for (int e = threadIdx.x; e < Nz * TL; e += blockDim.x) {
    const int row = e >> ltl, t = e & (TL - 1);
    const int l = l0 + t;
    const int pos = (row & 1) ? (Nz - 1 - (row >> 1)) : (row >> 1);
    if (l < lines) S[row * stride + l] = buf[(pos << ltl) + t];
  }
}

// ---- Navier-Stokes projection -------------------------------------------------------
// spec holds four fields of Nz*Ny*P complex each: r_u, r_v, r_w on entry (fields 0-2); on
// exit u^{n+1}, v^{n+1}, w^{n+1} and the pressure increment p' (field 3).
// WPE: waves per SIMD the registers must allow (two 1024-thread blocks per CU take 8).
template <typename T, int WPE>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(WPE)))
    k_zpass_ns(cx<T>* __restrict__ spec, int P, int Ny, int Nz, const double* __restrict__ lamx,
               const double* __restrict__ lamy, const double* __restrict__ phx,
               const double* __restrict__ phy, double ihx, double ihy, double ihz, double nu_m,
               double g_dt, double g_rho_dt, double scale, double4 wall) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int TL = blockDim.x / Nz;
  const int line = threadIdx.x % TL;
  const int row = threadIdx.x / TL;
  const int lines = P * Ny;
  const int l = xcd_block() * TL + line;
  const bool valid = l < lines;
  const int lc = valid ? l : lines - 1;
  int ky, kx;
  spec_mode(lc, P, Ny, ky, kx);
  const size_t stride = (size_t)lines;
  const size_t fsz = stride * Nz;
  const size_t at = row * stride + l;
  const double lxy = lamx[kx] + lamy[ky];
  const bool top = row == Nz - 1;
  const bool end = row == 0 || top;
  const T sc = (T)scale;
  // moving walls (eq. NS13): the no-slip ghosts of u and v carry 2 u_w, a layer constant in x
  // and y; moved to the right-hand side it is -nu_m 2 u_w / hz^2 on the wall rows of the (0,0)
  // mode (wall = that term for u at the bottom and top, v at the bottom and top)
  // ---- velocity Helmholtz (nu_m L - gamma0/dt) u~ = r: no-slip walls for u and v at cell
  // centres; w on z faces k = 0..Nz-2, the top-wall row an identity row. Both operators are
  // reduced together.
  const double av = nu_m * ihz * ihz;
  T a[2], b[2], c[2];
  cx<T> d[3];
  d[0] = valid ? sc * spec[at] : mk<T>(0, 0);
  d[1] = valid ? sc * spec[fsz + at] : mk<T>(0, 0);
  d[2] = (valid && !top) ? sc * spec[2 * fsz + at] : mk<T>(0, 0);
  if (l == 0 && end) {
    d[0].re += (T)(row == 0 ? wall.x : wall.y);
    d[1].re += (T)(row == 0 ? wall.z : wall.w);
  }
  a[0] = row == 0 ? (T)0 : (T)av;
  c[0] = top ? (T)0 : (T)av;
  b[0] = (T)(nu_m * lxy - (end ? 3.0 : 2.0) * av - g_dt);
  a[1] = (row == 0 || top) ? (T)0 : (T)av;
  c[1] = (row >= Nz - 2) ? (T)0 : (T)av;
  b[1] = top ? (T)1 : (T)(nu_m * lxy - 2.0 * av - g_dt);
  pcr_sym<T, 2, 3, 4>(smem, Nz, TL, row, line, a, b, c, d);
  if (top) d[2] = mk<T>(0, 0);
  // ---- divergence at centres: D_x = (1 - e^{-i th_x}) / hx, D_z w = (w_k - w_{k-1}) / hz
  cx<double>* Lw = reinterpret_cast<cx<double>*>(smem);
  const cx<double> u = widen<double>(d[0]), v = widen<double>(d[1]), wk = widen<double>(d[2]);
  Lw[row * TL + line] = wk;
  __syncthreads();
  const double cxr = phx[2 * kx], cxi = phx[2 * kx + 1];
  const double cyr = phy[2 * ky], cyi = phy[2 * ky + 1];
  const double dxr = (1.0 - cxr) * ihx, dxi = cxi * ihx;
  const double dyr = (1.0 - cyr) * ihy, dyi = cyi * ihy;
  const cx<double> wm = row > 0 ? Lw[(row - 1) * TL + line] : mk<double>(0, 0);
  cx<double> p[1];
  p[0] = mk<double>(g_rho_dt * (dxr * u.re - dxi * u.im + dyr * v.re - dyi * v.im + (wk.re - wm.re) * ihz),
                    g_rho_dt * (dxr * u.im + dxi * u.re + dyr * v.im + dyi * v.re + (wk.im - wm.im) * ihz));
  __syncthreads();
  // ---- FP64 Poisson (Neumann) for p'; the (0,0) mode is pinned at row 0, its mean removed
  const double ap = ihz * ihz;
  const bool pinned = kx == 0 && ky == 0;
  double pa[1] = {row == 0 ? 0.0 : ap}, pc[1] = {top ? 0.0 : ap}, pb[1] = {lxy - (end ? 1.0 : 2.0) * ap};
  if (pinned) {
    if (row == 0) { pa[0] = 0.0; pc[0] = 0.0; pb[0] = 1.0; p[0] = mk<double>(0, 0); }
    if (row == 1) pa[0] = 0.0;
  }
  pcr_sym<double, 1, 1, 0>(smem, Nz, TL, row, line, pa, pb, pc, p);
  cx<double>* Lp = reinterpret_cast<cx<double>*>(smem);
  Lp[row * TL + line] = p[0];
  __syncthreads();
  cx<double> pup = row < Nz - 1 ? Lp[(row + 1) * TL + line] : mk<double>(0, 0);
  if (pinned) {
    double mre = 0, mim = 0;
    for (int k = 0; k < Nz; ++k) {
      mre += Lp[k * TL + line].re;
      mim += Lp[k * TL + line].im;
    }
    mre /= Nz;
    mim /= Nz;
    p[0] = mk<double>(p[0].re - mre, p[0].im - mim);
    pup = mk<double>(pup.re - mre, pup.im - mim);
  }
  // ---- correction u = u~ - c grad p', G_x = (e^{i th_x} - 1) / hx
  const double cg = 1.0 / g_rho_dt;
  const double gxr = (cxr - 1.0) * ihx, gxi = cxi * ihx;
  const double gyr = (cyr - 1.0) * ihy, gyi = cyi * ihy;
  const double pr = p[0].re, pi = p[0].im;
  if (valid) {
    spec[at] = mk<T>((T)(u.re - cg * (gxr * pr - gxi * pi)), (T)(u.im - cg * (gxr * pi + gxi * pr)));
    spec[fsz + at] = mk<T>((T)(v.re - cg * (gyr * pr - gyi * pi)), (T)(v.im - cg * (gyr * pi + gyi * pr)));
    spec[2 * fsz + at] = top ? mk<T>(0, 0)
                             : mk<T>((T)(wk.re - cg * (pup.re - pr) * ihz), (T)(wk.im - cg * (pup.im - pi) * ihz));
    spec[3 * fsz + at] = mk<T>((T)pr, (T)pi);
  }
}

// ---- Navier-Stokes projection, transposed (FP64) --------------------------------------
// With Pi = I - G P+ D the projection (P+ the pseudo-inverse of the Neumann Laplacian, whose
// transpose is itself; G^T = -D with the top-wall w held at zero) and p^{n+1} = p^n + k P+ D u~
// (k = gamma0 rho0 / dt), the transpose maps (lam_u, lam_p) to
//   lam_u~ = lam_u - G P+ (D lam_u + k lam_p),
// and the velocity Helmholtz operators are symmetric, so lam_r = H^{-1} lam_u~ by the same
// per-mode solves. P+ discards the mean of its right-hand side (the (0,0) line's z-mean)
// before the pinned solve. spec holds lam_u, lam_v, lam_w, lam_p on entry and lam_r in the
// first three fields on exit.
__global__ void __launch_bounds__(1024)
    k_zpass_ns_adj(cx<double>* __restrict__ spec, int P, int Ny, int Nz, const double* __restrict__ lamx,
                   const double* __restrict__ lamy, const double* __restrict__ phx,
                   const double* __restrict__ phy, double ihx, double ihy, double ihz, double nu_m,
                   double g_dt, double g_rho_dt, double scale) {
  using T = double;
  extern __shared__ __align__(16) unsigned char smem[];
  const int TL = blockDim.x / Nz;
  const int line = threadIdx.x % TL;
  const int row = threadIdx.x / TL;
  const int lines = P * Ny;
  const int l = xcd_block() * TL + line;
  const bool valid = l < lines;
  const int lc = valid ? l : lines - 1;
  int ky, kx;
  spec_mode(lc, P, Ny, ky, kx);
  const size_t stride = (size_t)lines;
  const size_t fsz = stride * Nz;
  const size_t at = row * stride + l;
  const double lxy = lamx[kx] + lamy[ky];
  const bool end = row == 0 || row == Nz - 1;
  const bool top = row == Nz - 1;
  const cx<T> u = valid ? scale * spec[at] : mk<T>(0, 0);
  const cx<T> v = valid ? scale * spec[fsz + at] : mk<T>(0, 0);
  const cx<T> w = (valid && !top) ? scale * spec[2 * fsz + at] : mk<T>(0, 0);
  const cx<T> lp = valid ? scale * spec[3 * fsz + at] : mk<T>(0, 0);
  const double cxr = phx[2 * kx], cxi = phx[2 * kx + 1];
  const double cyr = phy[2 * ky], cyi = phy[2 * ky + 1];
  // ---- right-hand side D lam_u + k lam_p
  cx<T>* Ls = reinterpret_cast<cx<T>*>(smem);
  Ls[row * TL + line] = w;
  __syncthreads();
  const cx<T> wm = row > 0 ? Ls[(row - 1) * TL + line] : mk<T>(0, 0);
  const double dxr = (1.0 - cxr) * ihx, dxi = cxi * ihx;
  const double dyr = (1.0 - cyr) * ihy, dyi = cyi * ihy;
  cx<T> p[1];
  p[0] = mk<T>(dxr * u.re - dxi * u.im + dyr * v.re - dyi * v.im + (w.re - wm.re) * ihz + g_rho_dt * lp.re,
               dxr * u.im + dxi * u.re + dyr * v.im + dyi * v.re + (w.im - wm.im) * ihz + g_rho_dt * lp.im);
  __syncthreads();
  // ---- the (0,0) line: drop the z-mean of the right-hand side (pseudo-inverse)
  const bool pinned = kx == 0 && ky == 0;
  Ls[row * TL + line] = p[0];
  __syncthreads();
  if (pinned) {
    double mre = 0, mim = 0;
    for (int k = 0; k < Nz; ++k) {
      mre += Ls[k * TL + line].re;
      mim += Ls[k * TL + line].im;
    }
    p[0] = mk<T>(p[0].re - mre / Nz, p[0].im - mim / Nz);
  }
  __syncthreads();
  // ---- Poisson, pinned at row 0 for the (0,0) line, then its mean removed
  const double ap = ihz * ihz;
  double pa = row == 0 ? 0.0 : ap, pc = row == Nz - 1 ? 0.0 : ap;
  double pb = lxy - (end ? 1.0 : 2.0) * ap;
  if (pinned) {
    if (row == 0) { pa = 0.0; pc = 0.0; pb = 1.0; p[0] = mk<T>(0, 0); }
    if (row == 1) pa = 0.0;
  }
  {
    double pa1[1] = {pa}, pb1[1] = {pb}, pc1[1] = {pc};
    pcr_sym<double, 1, 1, 0>(smem, Nz, TL, row, line, pa1, pb1, pc1, p);
  }
  cx<T>* Lp = reinterpret_cast<cx<T>*>(smem);
  Lp[row * TL + line] = p[0];
  __syncthreads();
  cx<T> pup = row < Nz - 1 ? Lp[(row + 1) * TL + line] : mk<T>(0, 0);
  if (pinned) {
    double mre = 0, mim = 0;
    for (int k = 0; k < Nz; ++k) {
      mre += Lp[k * TL + line].re;
      mim += Lp[k * TL + line].im;
    }
    mre /= Nz;
    mim /= Nz;
    p[0] = mk<T>(p[0].re - mre, p[0].im - mim);
    pup = mk<T>(pup.re - mre, pup.im - mim);
  }
  __syncthreads();
  // ---- lam_u~ = lam_u - G q
  const double gxr = (cxr - 1.0) * ihx, gxi = cxi * ihx;
  const double gyr = (cyr - 1.0) * ihy, gyi = cyi * ihy;
  const double pr = p[0].re, pi = p[0].im;
  cx<T> uv[2];
  uv[0] = mk<T>(u.re - (gxr * pr - gxi * pi), u.im - (gxr * pi + gxi * pr));
  uv[1] = mk<T>(v.re - (gyr * pr - gyi * pi), v.im - (gyr * pi + gyi * pr));
  cx<T> wt[1];
  wt[0] = top ? mk<T>(0, 0) : mk<T>(w.re - (pup.re - pr) * ihz, w.im - (pup.im - pi) * ihz);
  // ---- velocity Helmholtz solves (the forward operators, symmetric), reduced together
  const double av = nu_m * ihz * ihz;
  T a[2] = {row == 0 ? 0.0 : av, (row == 0 || top) ? 0.0 : av};
  T b[2] = {nu_m * lxy - (end ? 3.0 : 2.0) * av - g_dt, top ? 1.0 : nu_m * lxy - 2.0 * av - g_dt};
  T c[2] = {row == Nz - 1 ? 0.0 : av, (row >= Nz - 2) ? 0.0 : av};
  cx<T> d[3] = {uv[0], uv[1], wt[0]};
  pcr_sym<T, 2, 3, 4>(smem, Nz, TL, row, line, a, b, c, d);
  uv[0] = d[0];
  uv[1] = d[1];
  wt[0] = top ? mk<T>(0, 0) : d[2];
  if (valid) {
    spec[at] = uv[0];
    spec[fsz + at] = uv[1];
    spec[2 * fsz + at] = wt[0];
  }
}

}  // namespace

template <typename T>
hipError_t launch_zpass_helmholtz(const Dims& d, const Tables<T>& tb, cx<T>* spec, int bc,
                                  double coeff, double shift, double scale, hipStream_t st) {
  const int lines = d.lines();
  const int TL = spread_lines(tile_lines(d.nz), lines, 2048);
  const size_t shm = pcr_sym_bytes<double, 1, 1>(d.nz, TL);
  hipLaunchKernelGGL(k_zpass_helmholtz<T>, dim3((lines + TL - 1) / TL), dim3(TL * d.nz), shm, st, spec,
                     d.pitch, d.ny, d.nz, tb.lam_x, tb.lam_y, 1.0 / (d.hz * d.hz), bc, coeff, shift,
                     scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wall_rhs(const Dims& d, int bc, double coeff, const T* rhs, const T* wall, T* out,
                           hipStream_t st) {
  const int layer = d.nx * d.ny;
  const double ihz = 1.0 / d.hz;
  // coefficient of the wall value in b (both walls alike), times coeff
  const double c = coeff * (bc == 0 ? ihz : bc == 1 ? 2.0 * ihz * ihz : ihz * ihz);
  const size_t n = (size_t)layer * d.nz;
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_wall_rhs<T>, dim3(blocks), dim3(256), 0, st, rhs, wall, out, layer, d.nz, bc, (T)c, (T)c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_top_layer(const Dims& d, const T* top, T* x, hipStream_t st) {
  const int layer = d.nx * d.ny;
  const int blocks = (layer + 255) / 256 < 1024 ? (layer + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_top_layer<T>, dim3(blocks), dim3(256), 0, st, top, x, layer, (size_t)(d.nz - 1) * layer);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zpass_ch(const Dims& d, const Tables<T>& tb, cx<T>* spec, double c_psi,
                           double alpha, double scale, double dwall, hipStream_t st, bool trans) {
  if (trans && (sizeof(T) != 8 || dwall == 0.0)) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 8) {
    // tiles of 128 bytes per row (8 complex FP64 modes): one cache line
    int TL = (int)(128 / sizeof(cx<T>));
    while (TL > 1 && TL * d.nz > 4096) TL >>= 1;
    TL = spread_lines(TL, d.lines(), 2048);
    int threads = TL * (d.nz >= 4 ? d.nz / 4 : 1);
    threads = ((threads + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    const int lines = d.lines();
    int lognz = 0;
    while ((1 << lognz) < d.nz) ++lognz;
    size_t shm = (size_t)d.nz * (TL + 1) * sizeof(cx<T>);
    // the inverse transforms are unnormalised: fold 1/nz into the spectral scale
    if (dwall == 0.0) {
      hipLaunchKernelGGL((k_zpass_ch_rt<T, false>), dim3((lines + TL - 1) / TL), dim3(threads), shm, st, spec,
                         d.pitch, d.ny, d.nz, lognz, TL, tb.lam_x, tb.lam_y, tb.lam_z, tb.tw_z, tb.tw_zq, c_psi,
                         alpha, scale / d.nz, 0.0);
    } else {
      // relaxed walls: partial sums (at most 16 per mode, 6 doubles each) and the wall sums
      const int nc = (threads / TL) < 16 ? threads / TL : 16;
      shm = ((shm + 15) & ~(size_t)15) + (size_t)2 * TL * sizeof(cx<double>) + (size_t)6 * nc * TL * sizeof(double) +
            (size_t)d.nz * TL * sizeof(T);
      auto kern = trans ? k_zpass_ch_rt<T, true, true> : k_zpass_ch_rt<T, true, false>;
      hipLaunchKernelGGL(kern, dim3((lines + TL - 1) / TL), dim3(threads), shm, st, spec, d.pitch, d.ny, d.nz,
                         lognz, TL, tb.lam_x, tb.lam_y, tb.lam_z, tb.tw_z, tb.tw_zq, c_psi, alpha, scale / d.nz,
                         dwall);
    }
    return hipGetLastError();
  } else {
    int lognz = 0;
    while ((1 << lognz) < d.nz) ++lognz;
    // tiles of 128 bytes per row (16 complex FP32 modes): one cache line; at most 4096 points
    // and kZBlock threads of P points per block
    int TL = 16;
    const int per_line = d.nz > (1 << fft_lp<T>()) ? d.nz >> fft_lp<T>() : 1;
    while (TL > 1 && (TL * d.nz > 4096 || TL * per_line > kZBlock)) TL >>= 1;
    TL = spread_lines(TL, d.lines(), 2048);
    const int lines = d.lines();
    const int threads = TL * per_line;
    // the inverse transforms are unnormalised: fold 1/nz into the spectral scale
    return with_logm(lognz, [&](auto L) {
      constexpr int LOGNZ = decltype(L)::value;
      using F = FftPlan<LOGNZ, fft_lp<T>()>;
      size_t shm = ((size_t)TL * F::LS + F::M) * sizeof(cx<T>);
      if (dwall == 0.0) {
        hipLaunchKernelGGL((k_zpass_ch<T, false, LOGNZ>), dim3((lines + TL - 1) / TL), dim3(threads), shm, st,
                           spec, d.pitch, d.ny, TL, tb.lam_x, tb.lam_y, tb.lam_z, tb.tw_z, tb.tw_zq, c_psi, alpha,
                           scale / d.nz, 0.0);
      } else {
        // relaxed walls: partial sums (at most 16 per mode, 6 doubles each) and the wall sums
        const int nc = (threads / TL) < 16 ? threads / TL : 16;
        shm = ((shm + 15) & ~(size_t)15) + (size_t)2 * TL * sizeof(cx<double>) + (size_t)6 * nc * TL * sizeof(double) +
              (size_t)d.nz * TL * sizeof(T);
        hipLaunchKernelGGL((k_zpass_ch<T, true, LOGNZ>), dim3((lines + TL - 1) / TL), dim3(threads), shm, st,
                           spec, d.pitch, d.ny, TL, tb.lam_x, tb.lam_y, tb.lam_z, tb.tw_z, tb.tw_zq, c_psi, alpha,
                           scale / d.nz, dwall);
      }
    });
  }
}

template <typename T>
hipError_t launch_zpass_ns(const Dims& d, const Tables<T>& tb, cx<T>* spec4, const StepConsts& c,
                           double scale, hipStream_t st) {
  const int lines = d.lines();
  auto shm_of = [&](int tl) {
    const size_t a = pcr_sym_bytes<T, 2, 3>(d.nz, tl), b = pcr_sym_bytes<double, 1, 1>(d.nz, tl);
    return a > b ? a : b;
  };
  // at most 64 KB of LDS per block (the FP64 form of a 1024-thread block would need 96 KB)
  int TL = tile_lines(d.nz);
  while (TL > 1 && shm_of(TL) > 65536) TL >>= 1;
  TL = spread_lines(TL, lines, 2048);
  const double bw = -2.0 * c.nu_m / (d.hz * d.hz);
  const double4 wall = make_double4(bw * c.uwb[0], bw * c.uwt[0], bw * c.uwb[1], bw * c.uwt[1]);
  // FP32: registers for two blocks of 1024 threads per CU; FP64 (whose LDS allows one such
  // block) unconstrained
  constexpr int WPE = sizeof(T) == 4 ? 8 : 4;
  hipLaunchKernelGGL((k_zpass_ns<T, WPE>), dim3((lines + TL - 1) / TL), dim3(TL * d.nz), shm_of(TL), st, spec4,
                     d.pitch, d.ny, d.nz, tb.lam_x, tb.lam_y, tb.ph_x, tb.ph_y, 1.0 / d.hx, 1.0 / d.hy,
                     1.0 / d.hz, c.nu_m, c.gamma0 / c.dt, c.gamma0 * c.rho0 / c.dt, scale, wall);
  return hipGetLastError();
}

hipError_t launch_zpass_ns_adj(const Dims& d, const Tables<double>& tb, cx<double>* spec4,
                               const StepConsts& c, double scale, hipStream_t st) {
  const int lines = d.lines();
  auto shm_of = [&](int tl) {
    const size_t a = pcr_sym_bytes<double, 2, 3>(d.nz, tl), b = pcr_sym_bytes<double, 1, 1>(d.nz, tl);
    return a > b ? a : b;
  };
  // at most 64 KB of LDS per block, as in the forward pass
  int TL = tile_lines(d.nz);
  while (TL > 1 && shm_of(TL) > 65536) TL >>= 1;
  TL = spread_lines(TL, lines, 2048);
  const size_t shm = shm_of(TL);
  hipLaunchKernelGGL(k_zpass_ns_adj, dim3((lines + TL - 1) / TL), dim3(TL * d.nz), shm, st, spec4, d.pitch,
                     d.ny, d.nz, tb.lam_x, tb.lam_y, tb.ph_x, tb.ph_y, 1.0 / d.hx, 1.0 / d.hy, 1.0 / d.hz,
                     c.nu_m, c.gamma0 / c.dt, c.gamma0 * c.rho0 / c.dt, scale);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_zpass_helmholtz<T>(const Dims&, const Tables<T>&, cx<T>*,  \
                                                int, double, double, double, hipStream_t);       \
  template hipError_t launch_wall_rhs<T>(const Dims&, int, double, const T*, const T*, T*,     \
                                         hipStream_t);                                          \
  template hipError_t launch_top_layer<T>(const Dims&, const T*, T*, hipStream_t);             \
  template hipError_t launch_zpass_ch<T>(const Dims&, const Tables<T>&, cx<T>*, double, \
                                         double, double, double, hipStream_t, bool);             \
  template hipError_t launch_zpass_ns<T>(const Dims&, const Tables<T>&, cx<T>*,         \
                                         const StepConsts&, double, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
