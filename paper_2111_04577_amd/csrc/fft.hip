// Batched FFT passes of the constant-coefficient solver (the "FFT solver" used for the
// Helmholtz and Poisson equations, Sec. 3.2.1-3.2.2 of the paper), written for gfx950:
// every line is staged in LDS, transformed there and written back with coalesced row
// accesses. FP32: lds_fft16.hpp (compile-time length, 8 points per thread, radix-8 Stockham
// stages with immediate LDS offsets); FP64: lds_fft.hpp (run-time length, radix-4, lanes on
// consecutive LDS words), the faster form for each element size.
//
//   x pass: real rows of length nx -> nx/2+1 complex (r2c through a length nx/2 complex
//           FFT of the even/odd-packed row), and the inverse (c2r). Unnormalised. Output in
//           the spectral layout of common.hpp (Nyquist modes of a layer stored apart).
//   y pass: complex columns of length ny, in place, on a tile of consecutive kx columns so
//           that each y-row load is contiguous and cache-line aligned; the Nyquist column of
//           a layer is one contiguous vector. Unnormalised.
#include "kernels.hpp"
#include "lds_fft.hpp"
#include "lds_fft16.hpp"

namespace drpf {

namespace {

constexpr int kBlock = 256;

// ---- x pass, forward (r2c) -------------------------------------------------------------
// A block holds lpb rows (FftPlan line layout), T = M / P threads per row.
template <typename T, int LOGM>
__global__ void __launch_bounds__(kBlock) k_fft_x_fwd(const T* __restrict__ in0,
                                                      const T* __restrict__ in1,
                                                      const T* __restrict__ in2,
                                                      cx<T>* __restrict__ out,
                                                      int lines_per_field, int total_lines,
                                                      int lpb, int Ny, const cx<T>* __restrict__ twM,
                                                      const cx<T>* __restrict__ twN) {
  using F = FftPlan<LOGM, fft_lp<T>()>;
  constexpr int M = F::M;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int line0 = blockIdx.x * lpb;
  const int nl = min(lpb, total_lines - line0);
  cx<T>* stw = buf + lpb * F::LS;  // twiddles of the length-M transform, staged in LDS
  for (int e = threadIdx.x; e < M; e += blockDim.x) stw[e] = twM[e];
  // a block never straddles two fields: lpb divides lines_per_field
  const int field = line0 / lines_per_field;
  const T* in = field == 0 ? in0 : (field == 1 ? in1 : in2);
  const T* src = in + (size_t)(line0 - field * lines_per_field) * (2 * M);
  // a row of 2M reals read as M (even, odd) pairs: rows start at even offsets of arrays
  // aligned to at least 16 bytes, so each pair is one aligned load
  for (int e = threadIdx.x; e < nl * M; e += blockDim.x)
    buf[(e >> LOGM) * F::LS + F::pad(e & (M - 1))] = reinterpret_cast<const cx<T>*>(src)[e];
  __syncthreads();
  {
    const int b = threadIdx.x >> F::LT, q = threadIdx.x & (F::T - 1);
    fft16<T, false, LOGM, fft_lp<T>()>(buf + b * F::LS, q, b < nl, stw);
  }
  // row r = z Ny + ky of this field
  const size_t lines = (size_t)(M + 1) * Ny;
  cx<T>* fbase = out + (size_t)field * lines * (lines_per_field / Ny);
  const int r0 = line0 - field * lines_per_field;
  const int lny = __ffs(Ny) - 1;
  const T half = (T)0.5;
  auto mode = [&](int b, int k) {
    const cx<T>* row = buf + b * F::LS;
    const cx<T> zk = row[F::pad(k == M ? 0 : k)];
    const cx<T> zm = conj(row[F::pad(k == 0 ? 0 : M - k)]);
    const cx<T> E = half * (zk + zm);
    const cx<T> O = half * mul_mi(zk - zm);
    return E + twN[k] * O;
  };
  // modes k < M, then the Nyquist mode of every row
  for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
    const int b = e >> LOGM, k = e & (M - 1);
    const int r = r0 + b, z = r >> lny, ky = r & (Ny - 1);
    fbase[z * lines + (size_t)ky * M + k] = mode(b, k);
  }
  for (int b = threadIdx.x; b < nl; b += blockDim.x) {
    const int r = r0 + b, z = r >> lny, ky = r & (Ny - 1);
    fbase[z * lines + (size_t)M * Ny + ky] = mode(b, M);
  }
}

// ---- x pass, inverse (c2r), up to four output fields with optional addend --------------
template <typename T, int LOGM>
__global__ void __launch_bounds__(kBlock) k_fft_x_inv(const cx<T>* __restrict__ in, RealSet<T> out,
                                                      int lines_per_field, int total_lines, int lpb,
                                                      int Ny, const cx<T>* __restrict__ twM,
                                                      const cx<T>* __restrict__ twN) {
  using F = FftPlan<LOGM, fft_lp<T>()>;
  constexpr int M = F::M;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int line0 = blockIdx.x * lpb;
  const int nl = min(lpb, total_lines - line0);
  cx<T>* stw = buf + lpb * F::LS;
  for (int e = threadIdx.x; e < M; e += blockDim.x) stw[e] = twM[e];
  const int field0 = line0 / lines_per_field;
  const size_t lines = (size_t)(M + 1) * Ny;
  const cx<T>* fbase = in + (size_t)field0 * lines * (lines_per_field / Ny);
  const int r0 = line0 - field0 * lines_per_field;
  const int lny = __ffs(Ny) - 1;
  for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
    const int b = e >> LOGM;
    const int k = e & (M - 1);
    const int r = r0 + b, z = r >> lny, ky = r & (Ny - 1);
    const cx<T>* src = fbase + z * lines;
    const cx<T> xk = src[(size_t)ky * M + k];
    const cx<T> xm = conj(k == 0 ? src[(size_t)M * Ny + ky] : src[(size_t)ky * M + (M - k)]);
    const cx<T> E = xk + xm;
    const cx<T> O = conj(twN[k]) * (xk - xm);
    buf[b * F::LS + F::pad(k)] = E + mul_i(O);
  }
  __syncthreads();
  {
    const int b = threadIdx.x >> F::LT, q = threadIdx.x & (F::T - 1);
    fft16<T, true, LOGM, fft_lp<T>()>(buf + b * F::LS, q, b < nl, stw);
  }
  const int field = line0 / lines_per_field;
  T* dst = out.p[field] + (size_t)(line0 - field * lines_per_field) * (2 * M);
  const T* add = out.add[field];
  if (add != nullptr) {
    add += (size_t)(line0 - field * lines_per_field) * (2 * M);
    for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
      const cx<T> a = reinterpret_cast<const cx<T>*>(add)[e];
      const cx<T> v = buf[(e >> LOGM) * F::LS + F::pad(e & (M - 1))];
      reinterpret_cast<cx<T>*>(dst)[e] = mk<T>(a.re + v.re, a.im + v.im);
    }
  } else {
    for (int e = threadIdx.x; e < nl * M; e += blockDim.x)
      reinterpret_cast<cx<T>*>(dst)[e] = buf[(e >> LOGM) * F::LS + F::pad(e & (M - 1))];
  }
}

// ---- y pass (c2c, in place) -------------------------------------------------------------
// A block holds tkx columns of one batch as lines of length Ny = 2^LOGY.
template <typename T, bool INV, int LOGY>
__global__ void __launch_bounds__(1024) k_fft_y(cx<T>* __restrict__ data, int P, int ntiles, int tkx,
                                                  const cx<T>* __restrict__ tw) {
  using F = FftPlan<LOGY, fft_lp<T>()>;
  constexpr int Ny = F::M;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int M = P - 1;
  // XCD-ordered: consecutive tiles, which share cache lines when a tile row is narrower than a
  // line (FP32 tiles of 8 modes, 64 bytes, on 512-point lines), run on one XCD and its L2
  const int lb = xcd_block();
  const int tile = lb % ntiles;
  const int batch = lb / ntiles;
  cx<T>* base = data + (size_t)batch * Ny * P;
  // tiles 0 .. ntiles-2: tkx consecutive kx < M of every row; the last tile: the Nyquist
  // column (contiguous in ky), as line 0 of the tile
  const bool nyq = tile == ntiles - 1;
  const int kx0 = tile * tkx;
  cx<T>* stw = buf + tkx * F::LS;
  const int ltk = __ffs(tkx) - 1;  // tkx is a power of two
  for (int e = threadIdx.x; e < Ny; e += blockDim.x) stw[e] = tw[e];
  const int nl = nyq ? 1 : tkx;
  for (int e = threadIdx.x; e < Ny * nl; e += blockDim.x) {
    if (nyq) {
      buf[F::pad(e)] = base[(size_t)M * Ny + e];
    } else {
      const int y = e >> ltk, t = e & (tkx - 1);
      buf[t * F::LS + F::pad(y)] = base[(size_t)y * M + kx0 + t];
    }
  }
  __syncthreads();
  {
    const int b = threadIdx.x >> F::LT, q = threadIdx.x & (F::T - 1);
    fft16<T, INV, LOGY, fft_lp<T>()>(buf + b * F::LS, q, b < nl, stw);
  }
  for (int e = threadIdx.x; e < Ny * nl; e += blockDim.x) {
    if (nyq) {
      base[(size_t)M * Ny + e] = buf[F::pad(e)];
    } else {
      const int y = e >> ltk, t = e & (tkx - 1);
      base[(size_t)y * M + kx0 + t] = buf[t * F::LS + F::pad(y)];
    }
  }
}

// ---- run-time length forms (the FP64 passes) --------------------------------------------
// Every line is transformed by lds_fft (radix-4 Stockham, one butterfly set per thread).

// ---- x pass, forward (r2c), run-time length ----------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fft_x_fwd_rt(const T* __restrict__ in0,
                                                      const T* __restrict__ in1,
                                                      const T* __restrict__ in2,
                                                      cx<T>* __restrict__ out, int N, int logM,
                                                      int lines_per_field, int total_lines,
                                                      int lpb, int Ny, const cx<T>* __restrict__ twM,
                                                      const cx<T>* __restrict__ twN) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int M = N >> 1;
  const int line0 = blockIdx.x * lpb;
  const int nl = min(lpb, total_lines - line0);
  cx<T>* stw = buf + lpb * M;  // twiddles of the length-M transform, staged in LDS
  for (int e = threadIdx.x; e < M; e += blockDim.x) stw[e] = twM[e];
  // a block never straddles two fields: lpb divides lines_per_field
  const int field = line0 / lines_per_field;
  const T* in = field == 0 ? in0 : (field == 1 ? in1 : in2);
  const T* src = in + (size_t)(line0 - field * lines_per_field) * N;
  // a row of N reals read as N/2 (even, odd) pairs: rows start at even offsets of arrays
  // aligned to at least 16 bytes, so each pair is one aligned load
  for (int e = threadIdx.x; e < nl * M; e += blockDim.x) buf[e] = reinterpret_cast<const cx<T>*>(src)[e];
  __syncthreads();
  lds_fft<T, false, false>(buf, M, logM, nl, 0, stw);
  // row r = z Ny + ky of this field
  const size_t lines = (size_t)(M + 1) * Ny;
  cx<T>* fbase = out + (size_t)field * lines * (lines_per_field / Ny);
  const int r0 = line0 - field * lines_per_field;
  const int lny = __ffs(Ny) - 1;
  const T half = (T)0.5;
  auto mode = [&](int b, int k) {
    const cx<T> zk = buf[(b << logM) + (k == M ? 0 : k)];
    const cx<T> zm = conj(buf[(b << logM) + (k == 0 ? 0 : M - k)]);
    const cx<T> E = half * (zk + zm);
    const cx<T> O = half * mul_mi(zk - zm);
    return E + twN[k] * O;
  };
  // modes k < M, then the Nyquist mode of every row
  for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
    const int b = e >> logM, k = e & (M - 1);
    const int r = r0 + b, z = r >> lny, ky = r & (Ny - 1);
    fbase[z * lines + (size_t)ky * M + k] = mode(b, k);
  }
  for (int b = threadIdx.x; b < nl; b += blockDim.x) {
    const int r = r0 + b, z = r >> lny, ky = r & (Ny - 1);
    fbase[z * lines + (size_t)M * Ny + ky] = mode(b, M);
  }
}

// ---- x pass, inverse (c2r), run-time length --------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fft_x_inv_rt(const cx<T>* __restrict__ in, RealSet<T> out,
                                                      int N, int logM, int lines_per_field,
                                                      int total_lines, int lpb, int Ny,
                                                      const cx<T>* __restrict__ twM,
                                                      const cx<T>* __restrict__ twN) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int M = N >> 1;
  const int line0 = blockIdx.x * lpb;
  const int nl = min(lpb, total_lines - line0);
  cx<T>* stw = buf + lpb * M;
  for (int e = threadIdx.x; e < M; e += blockDim.x) stw[e] = twM[e];
  const int field0 = line0 / lines_per_field;
  const size_t lines = (size_t)(M + 1) * Ny;
  const cx<T>* fbase = in + (size_t)field0 * lines * (lines_per_field / Ny);
  const int r0 = line0 - field0 * lines_per_field;
  const int lny = __ffs(Ny) - 1;
  for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
    const int b = e >> logM;
    const int k = e & (M - 1);
    const int r = r0 + b, z = r >> lny, ky = r & (Ny - 1);
    const cx<T>* src = fbase + z * lines;
    const cx<T> xk = src[(size_t)ky * M + k];
    const cx<T> xm = conj(k == 0 ? src[(size_t)M * Ny + ky] : src[(size_t)ky * M + (M - k)]);
    const cx<T> E = xk + xm;
    const cx<T> O = conj(twN[k]) * (xk - xm);
    buf[e] = E + mul_i(O);
  }
  __syncthreads();
  lds_fft<T, true, false>(buf, M, logM, nl, 0, stw);
  const int field = line0 / lines_per_field;
  T* dst = out.p[field] + (size_t)(line0 - field * lines_per_field) * N;
  const T* add = out.add[field];
  if (add != nullptr) {
    add += (size_t)(line0 - field * lines_per_field) * N;
    for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
      const cx<T> a = reinterpret_cast<const cx<T>*>(add)[e];
      reinterpret_cast<cx<T>*>(dst)[e] = mk<T>(a.re + buf[e].re, a.im + buf[e].im);
    }
  } else {
    for (int e = threadIdx.x; e < nl * M; e += blockDim.x) reinterpret_cast<cx<T>*>(dst)[e] = buf[e];
  }
}

// ---- y pass (c2c, in place), run-time length ----------------------------------------
template <typename T, bool INV>
__global__ void k_fft_y_rt(cx<T>* __restrict__ data, int Ny, int logNy, int P, int ntiles, int tkx,
                        const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int M = P - 1;
  // XCD-ordered: consecutive tiles, which share cache lines when a tile row is narrower than a
  // line (FP32 tiles of 8 modes, 64 bytes, on 512-point lines), run on one XCD and its L2
  const int lb = xcd_block();
  const int tile = lb % ntiles;
  const int batch = lb / ntiles;
  cx<T>* base = data + (size_t)batch * Ny * P;
  // tiles 0 .. ntiles-2: tkx consecutive kx < M of every row; the last tile: the Nyquist
  // column (contiguous in ky), in lane 0 of the tile
  const bool nyq = tile == ntiles - 1;
  const int kx0 = tile * tkx;
  cx<T>* stw = buf + Ny * tkx;
  const int ltk = __ffs(tkx) - 1;  // tkx is a power of two
  for (int e = threadIdx.x; e < Ny; e += blockDim.x) stw[e] = tw[e];
  for (int e = threadIdx.x; e < Ny * tkx; e += blockDim.x) {
    const int y = e >> ltk;
    const int t = e & (tkx - 1);
    if (nyq)
      buf[e] = t == 0 ? base[(size_t)M * Ny + y] : mk<T>(0, 0);
    else
      buf[e] = base[(size_t)y * M + kx0 + t];
  }
  __syncthreads();
  lds_fft<T, INV, true>(buf, Ny, logNy, tkx, ltk, stw);
  for (int e = threadIdx.x; e < Ny * tkx; e += blockDim.x) {
    const int y = e >> ltk;
    const int t = e & (tkx - 1);
    if (nyq) {
      if (t == 0) base[(size_t)M * Ny + y] = buf[e];
    } else {
      base[(size_t)y * M + kx0 + t] = buf[e];
    }
  }
}

// ---- x and y passes together, one block per layer of one field --------------------------
// A whole layer (ny rows of nx reals; M = nx/2) in LDS: [ny][M] complex plus the Nyquist
// column. Forward: the half-length x transform of every row, the r2c split in place (pairs k
// and M - k, k = 0 giving mode 0 and the Nyquist mode), then the y transform of every column
// and of the Nyquist column, written in the spectral layout. The inverse runs the same steps
// backwards, with the addend of the real output. The same arithmetic as the separate passes,
// without the spectral round trip between them; used where a layer fits in a block's LDS.
template <typename T, int REP>
__global__ void __launch_bounds__(1024)
    k_fft_xy_fwd(const T* __restrict__ in0, const T* __restrict__ in1, const T* __restrict__ in2,
                 cx<T>* __restrict__ out, int N, int logM, int Ny, int logNy, int nz,
                 const cx<T>* __restrict__ twM, const cx<T>* __restrict__ twN,
                 const cx<T>* __restrict__ twY) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int M = N >> 1;
  cx<T>* A = reinterpret_cast<cx<T>*>(smem_raw);  // [Ny][M]
  cx<T>* Q = A + (Ny << logM);                     // Nyquist column [Ny]
  cx<T>* sM = Q + Ny;                              // x twiddles [M]
  cx<T>* sY = sM + M;                              // y twiddles [Ny]
  const int field = blockIdx.x / nz, z = blockIdx.x - field * nz;
  const T* in = field == 0 ? in0 : (field == 1 ? in1 : in2);
  const T* src = in + (size_t)z * Ny * N;
  for (int e = threadIdx.x; e < M; e += blockDim.x) sM[e] = twM[e];
  for (int e = threadIdx.x; e < Ny; e += blockDim.x) sY[e] = twY[e];
  const int n = Ny << logM;
  for (int e = threadIdx.x; e < n; e += blockDim.x) A[e] = reinterpret_cast<const cx<T>*>(src)[e];
  __syncthreads();
  lds_fft_rep<T, false, false, REP>(A, M, logM, Ny, 0, sM);
  const int half = M >> 1;
  const T hf = (T)0.5;
  // mode k from z_k and conj(z_{M-k}) of the half-length transform
  auto split = [&](cx<T> zk, cx<T> zmc, int k) {
    const cx<T> E = hf * (zk + zmc);
    const cx<T> O = hf * mul_mi(zk - zmc);
    return E + twN[k] * O;
  };
  // pairs k < half of every row (shifts and masks), then k = half of every row
  const int lh = logM - 1, nmain = Ny << lh;
  for (int e = threadIdx.x; e < nmain + Ny; e += blockDim.x) {
    const bool mid = e >= nmain;
    const int y = mid ? e - nmain : e >> lh, k = mid ? half : e & (half - 1);
    cx<T>* row = A + (y << logM);
    if (k == 0) {
      const cx<T> a = row[0];
      row[0] = split(a, conj(a), 0);
      Q[y] = split(a, conj(a), M);
    } else if (k == half) {
      const cx<T> a = row[half];
      row[half] = split(a, conj(a), half);
    } else {
      const cx<T> a = row[k], b = row[M - k];
      row[k] = split(a, conj(b), k);
      row[M - k] = split(b, conj(a), M - k);
    }
  }
  __syncthreads();
  lds_fft_rep<T, false, true, REP, true>(A, Ny, logNy, M, logM, sY, Q);
  const size_t lines = (size_t)(M + 1) * Ny;
  cx<T>* dst = out + (size_t)field * lines * nz + (size_t)z * lines;
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = A[e];
  for (int e = threadIdx.x; e < Ny; e += blockDim.x) dst[(size_t)M * Ny + e] = Q[e];
}

template <typename T, int REP>
__global__ void __launch_bounds__(1024)
    k_fft_xy_inv(const cx<T>* __restrict__ in, RealSet<T> out, int N, int logM, int Ny, int logNy,
                 int nz, const cx<T>* __restrict__ twM, const cx<T>* __restrict__ twN,
                 const cx<T>* __restrict__ twY) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int M = N >> 1;
  cx<T>* A = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* Q = A + (Ny << logM);
  cx<T>* sM = Q + Ny;
  cx<T>* sY = sM + M;
  const int field = blockIdx.x / nz, z = blockIdx.x - field * nz;
  const size_t lines = (size_t)(M + 1) * Ny;
  const cx<T>* src = in + (size_t)field * lines * nz + (size_t)z * lines;
  for (int e = threadIdx.x; e < M; e += blockDim.x) sM[e] = twM[e];
  for (int e = threadIdx.x; e < Ny; e += blockDim.x) sY[e] = twY[e];
  const int n = Ny << logM;
  for (int e = threadIdx.x; e < n; e += blockDim.x) A[e] = src[e];
  for (int e = threadIdx.x; e < Ny; e += blockDim.x) Q[e] = src[(size_t)M * Ny + e];
  __syncthreads();
  lds_fft_rep<T, true, true, REP, true>(A, Ny, logNy, M, logM, sY, Q);
  // c2r: z_k = E + i O, E = X_k + conj(X_{M-k}), O = conj(w_k)(X_k - conj(X_{M-k})), with
  // X_{M-0} read as the Nyquist mode
  const int half = M >> 1;
  auto join = [&](cx<T> xk, cx<T> xmc, int k) {
    const cx<T> E = xk + xmc;
    const cx<T> O = conj(twN[k]) * (xk - xmc);
    return E + mul_i(O);
  };
  // pairs k < half of every row (shifts and masks), then k = half of every row
  const int lh = logM - 1, nmain = Ny << lh;
  for (int e = threadIdx.x; e < nmain + Ny; e += blockDim.x) {
    const bool mid = e >= nmain;
    const int y = mid ? e - nmain : e >> lh, k = mid ? half : e & (half - 1);
    cx<T>* row = A + (y << logM);
    if (k == 0) {
      row[0] = join(row[0], conj(Q[y]), 0);
    } else if (k == half) {
      const cx<T> a = row[half];
      row[half] = join(a, conj(a), half);
    } else {
      const cx<T> a = row[k], b = row[M - k];
      row[k] = join(a, conj(b), k);
      row[M - k] = join(b, conj(a), M - k);
    }
  }
  __syncthreads();
  lds_fft_rep<T, true, false, REP>(A, M, logM, Ny, 0, sM);
  T* dst = out.p[field] + (size_t)z * Ny * N;
  const T* add = out.add[field];
  if (add != nullptr) {
    add += (size_t)z * Ny * N;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const cx<T> a = reinterpret_cast<const cx<T>*>(add)[e];
      reinterpret_cast<cx<T>*>(dst)[e] = mk<T>(a.re + A[e].re, a.im + A[e].im);
    }
  } else {
    for (int e = threadIdx.x; e < n; e += blockDim.x) reinterpret_cast<cx<T>*>(dst)[e] = A[e];
  }
}

int largest_pow2_divisor(int n, int cap) {
  int d = 1;
  while (d * 2 <= cap && n % (d * 2) == 0) d *= 2;
  return d;
}

// rows per block of the FP32 x passes: kBlock threads of T = M / P each, dividing the rows of
// a field
int x_lines_per_block16(int logm, int lpf) {
  const int lt = logm > fft_lp<float>() ? logm - fft_lp<float>() : 0;
  const int cap = (kBlock >> lt) >= 1 ? (kBlock >> lt) : 1;
  return largest_pow2_divisor(lpf, cap);
}

// rows per block of the run-time length x passes: one butterfly set of M/4 per thread
int x_lines_per_block(int M) {
  const int quarter = M >= 4 ? M / 4 : 1;
  return kBlock / quarter;  // M <= 1024 keeps this >= 1
}

}  // namespace

template <typename T>
hipError_t launch_fft_x_fwd(const Dims& d, const Tables<T>& tb, const T* const in[4], int nfields,
                            cx<T>* spec, hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    const int M = d.nx / 2;
    const int lpf = d.ny * d.nz;
    const int lpb = largest_pow2_divisor(lpf, x_lines_per_block(M));
    const int total = lpf * nfields;
    const int blocks = total / lpb;
    const size_t shm = (size_t)(lpb + 1) * M * sizeof(cx<T>);
    hipLaunchKernelGGL(k_fft_x_fwd_rt<T>, dim3(blocks), dim3(kBlock), shm, st, in[0],
                       nfields > 1 ? in[1] : in[0], nfields > 2 ? in[2] : in[0], spec, d.nx,
                       d.logx - 1, lpf, total, lpb, d.ny, tb.tw_xm, tb.tw_xn);
    return hipGetLastError();
  } else {
    const int logm = d.logx - 1;
    const int lpf = d.ny * d.nz;
    const int lpb = x_lines_per_block16(logm, lpf);
    const int total = lpf * nfields;
    const int blocks = total / lpb;
    return with_logm(logm, [&](auto L) {
      constexpr int LOGM = decltype(L)::value;
      using F = FftPlan<LOGM, fft_lp<T>()>;
      const size_t shm = ((size_t)lpb * F::LS + F::M) * sizeof(cx<T>);
      hipLaunchKernelGGL((k_fft_x_fwd<T, LOGM>), dim3(blocks), dim3(lpb * F::T), shm, st, in[0],
                         nfields > 1 ? in[1] : in[0], nfields > 2 ? in[2] : in[0], spec, lpf, total, lpb,
                         d.ny, tb.tw_xm, tb.tw_xn);
    });
  }
}

template <typename T>
hipError_t launch_fft_x_inv(const Dims& d, const Tables<T>& tb, const cx<T>* spec, RealSet<T> out,
                            hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    const int M = d.nx / 2;
    const int lpf = d.ny * d.nz;
    const int lpb = largest_pow2_divisor(lpf, x_lines_per_block(M));
    const int total = lpf * out.nfields;
    const int blocks = total / lpb;
    const size_t shm = (size_t)(lpb + 1) * M * sizeof(cx<T>);
    hipLaunchKernelGGL(k_fft_x_inv_rt<T>, dim3(blocks), dim3(kBlock), shm, st, spec, out, d.nx,
                       d.logx - 1, lpf, total, lpb, d.ny, tb.tw_xm, tb.tw_xn);
    return hipGetLastError();
  } else {
    const int logm = d.logx - 1;
    const int lpf = d.ny * d.nz;
    const int lpb = x_lines_per_block16(logm, lpf);
    const int total = lpf * out.nfields;
    const int blocks = total / lpb;
    return with_logm(logm, [&](auto L) {
      constexpr int LOGM = decltype(L)::value;
      using F = FftPlan<LOGM, fft_lp<T>()>;
      const size_t shm = ((size_t)lpb * F::LS + F::M) * sizeof(cx<T>);
      hipLaunchKernelGGL((k_fft_x_inv<T, LOGM>), dim3(blocks), dim3(lpb * F::T), shm, st, spec, out, lpf,
                         total, lpb, d.ny, tb.tw_xm, tb.tw_xn);
    });
  }
}

// LDS of one layer in the fused x-y passes, and the butterfly sets per thread (1024 threads)
template <typename T>
size_t fft_xy_lds(const Dims& d) {
  return ((size_t)(d.nx / 2) * d.ny + 2 * (size_t)d.ny + d.nx / 2) * sizeof(cx<T>);
}
int fft_xy_rep(const Dims& d) {
  const int M = d.nx / 2;
  const int sx = (M >= 4 ? M / 4 : 1) * d.ny, sy = (d.ny >= 4 ? d.ny / 4 : 1) * M;
  const int sets = sx > sy ? sx : sy;
  return sets <= 2048 ? 2 : (sets <= 4096 ? 4 : 0);
}

template <typename T>
bool fft_xy_fits(const Dims& d) {
  return d.ny > 1 && fft_xy_lds<T>(d) <= (size_t)160 * 1024 && fft_xy_rep(d) != 0;
}

template <typename T>
hipError_t launch_fft_xy_fwd(const Dims& d, const Tables<T>& tb, const T* const in[4], int nfields,
                             cx<T>* spec, hipStream_t st) {
  if (!fft_xy_fits<T>(d)) return hipErrorInvalidConfiguration;
  const size_t shm = fft_xy_lds<T>(d);
  const dim3 grid(nfields * d.nz), block(1024);
  const T* i1 = nfields > 1 ? in[1] : in[0];
  const T* i2 = nfields > 2 ? in[2] : in[0];
  if (fft_xy_rep(d) == 2)
    hipLaunchKernelGGL((k_fft_xy_fwd<T, 2>), grid, block, shm, st, in[0], i1, i2, spec, d.nx, d.logx - 1,
                       d.ny, d.logy, d.nz, tb.tw_xm, tb.tw_xn, tb.tw_y);
  else
    hipLaunchKernelGGL((k_fft_xy_fwd<T, 4>), grid, block, shm, st, in[0], i1, i2, spec, d.nx, d.logx - 1,
                       d.ny, d.logy, d.nz, tb.tw_xm, tb.tw_xn, tb.tw_y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_xy_inv(const Dims& d, const Tables<T>& tb, const cx<T>* spec, RealSet<T> out,
                             hipStream_t st) {
  if (!fft_xy_fits<T>(d)) return hipErrorInvalidConfiguration;
  const size_t shm = fft_xy_lds<T>(d);
  const dim3 grid(out.nfields * d.nz), block(1024);
  if (fft_xy_rep(d) == 2)
    hipLaunchKernelGGL((k_fft_xy_inv<T, 2>), grid, block, shm, st, spec, out, d.nx, d.logx - 1, d.ny,
                       d.logy, d.nz, tb.tw_xm, tb.tw_xn, tb.tw_y);
  else
    hipLaunchKernelGGL((k_fft_xy_inv<T, 4>), grid, block, shm, st, spec, out, d.nx, d.logx - 1, d.ny,
                       d.logy, d.nz, tb.tw_xm, tb.tw_xn, tb.tw_y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y(const Dims& d, const Tables<T>& tb, cx<T>* spec, int nfields, bool inverse,
                        hipStream_t st) {
  if (d.ny == 1) return hipSuccess;
  if constexpr (sizeof(T) == 8) {
    const int Ny = d.ny;
    // tiles of 128 bytes per row (8 complex FP64 columns): one cache line
    int tkx = (int)(128 / sizeof(cx<T>));
    while (tkx > 1 && tkx * Ny > 4096) tkx >>= 1;  // tkx * Ny / 4 <= 1024 threads
    while (tkx > d.nx / 2) tkx >>= 1;
    const int P = d.pitch;
    const int ntiles = (d.nx / 2) / tkx + 1;  // kx < nx/2 in tiles of tkx, then the Nyquist column
    const int batches = d.nz * nfields;
    int threads = tkx * (Ny >= 4 ? Ny / 4 : 1);
    threads = ((threads + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    const size_t shm = (size_t)Ny * (tkx + 1) * sizeof(cx<T>);
    if (inverse)
      hipLaunchKernelGGL((k_fft_y_rt<T, true>), dim3(ntiles * batches), dim3(threads), shm, st, spec, Ny,
                         d.logy, P, ntiles, tkx, tb.tw_y);
    else
      hipLaunchKernelGGL((k_fft_y_rt<T, false>), dim3(ntiles * batches), dim3(threads), shm, st, spec, Ny,
                         d.logy, P, ntiles, tkx, tb.tw_y);
    return hipGetLastError();
  } else {
    // tiles of 128 bytes per row (16 complex FP32 columns): one cache line, at most 4096 points
    // and 1024 threads of P points per block
    int tkx = 16;
    const int per_line = d.ny > (1 << fft_lp<T>()) ? d.ny >> fft_lp<T>() : 1;
    while (tkx > 1 && (tkx * d.ny > 4096 || tkx * per_line > 1024)) tkx >>= 1;
    while (tkx > d.nx / 2) tkx >>= 1;
    const int P = d.pitch;
    const int ntiles = (d.nx / 2) / tkx + 1;  // kx < nx/2 in tiles of tkx, then the Nyquist column
    const int batches = d.nz * nfields;
    return with_logm(d.logy, [&](auto L) {
      constexpr int LOGY = decltype(L)::value;
      using F = FftPlan<LOGY, fft_lp<T>()>;
      const size_t shm = ((size_t)tkx * F::LS + F::M) * sizeof(cx<T>);
      const dim3 grid(ntiles * batches), block(tkx * F::T);
      if (inverse)
        hipLaunchKernelGGL((k_fft_y<T, true, LOGY>), grid, block, shm, st, spec, P, ntiles, tkx, tb.tw_y);
      else
        hipLaunchKernelGGL((k_fft_y<T, false, LOGY>), grid, block, shm, st, spec, P, ntiles, tkx, tb.tw_y);
    });
  }
}

#define INST(T)                                                                                    \
  template hipError_t launch_fft_x_fwd<T>(const Dims&, const Tables<T>&, const T* const[4], int,   \
                                          cx<T>*, hipStream_t);                                    \
  template hipError_t launch_fft_x_inv<T>(const Dims&, const Tables<T>&, const cx<T>*, RealSet<T>, \
                                          hipStream_t);                                            \
  template hipError_t launch_fft_y<T>(const Dims&, const Tables<T>&, cx<T>*, int, bool, hipStream_t); \
  template bool fft_xy_fits<T>(const Dims&);                                                        \
  template hipError_t launch_fft_xy_fwd<T>(const Dims&, const Tables<T>&, const T* const[4], int,  \
                                           cx<T>*, hipStream_t);                                   \
  template hipError_t launch_fft_xy_inv<T>(const Dims&, const Tables<T>&, const cx<T>*, RealSet<T>, \
                                           hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace drpf
