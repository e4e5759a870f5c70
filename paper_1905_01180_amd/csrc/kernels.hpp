// Small kernels of the GKBA collision-integral path: matrix exponential,
// GKBA two-time slices, layout preparation of the interaction tensor, packing
// of the per-chunk operands, reductions.  The bulk contractions live in gemm.hpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm.hpp"

namespace sb2 {

typedef double cplx __attribute__((ext_vector_type(2)));   // (re, im)

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  cplx r;
  r[0] = a[0] * b[0] - a[1] * b[1];
  r[1] = a[0] * b[1] + a[1] * b[0];
  return r;
}
__device__ __forceinline__ cplx mk(double re, double im) {
  cplx r;
  r[0] = re;
  r[1] = im;
  return r;
}
__device__ __forceinline__ cplx conj_(cplx a) { return mk(a[0], -a[1]); }
__device__ __forceinline__ cplx times_i(cplx a) { return mk(-a[1], a[0]); }       // i a
__device__ __forceinline__ cplx times_mi(cplx a) { return mk(a[1], -a[0]); }      // -i a

__global__ void k_fill_u32(unsigned* p, int n, unsigned val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

// Optional input checks (SB2_CHECK=1).  out[0] is raised to max |X_ij -
// conj(X_ji)| over the nmat N x N matrices, out[1] to max |X_ij| (float bits of
// non-negative values), out[2] is set when any entry is not finite.
__global__ void k_check_herm(int N, i64 nmat, const cplx* __restrict__ X, unsigned* out) {
  const i64 nn = (i64)N * N;
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nmat * nn) return;
  const i64 m = idx / nn;
  const int i = (int)((idx - m * nn) / N), j = (int)(idx - m * nn - (i64)i * N);
  const cplx a = X[idx], b = X[m * nn + (i64)j * N + i];
  if (!isfinite(a[0]) || !isfinite(a[1])) {
    atomicOr(out + 2, 1u);
    return;
  }
  const double d = fmax(fabs(a[0] - b[0]), fabs(a[1] + b[1]));
  const double x = fmax(fabs(a[0]), fabs(a[1]));
  if (d > 0.0) atomicMax(out, __float_as_uint((float)d));
  if (x > 0.0) atomicMax(out + 1, __float_as_uint((float)x));
}

__global__ void k_check_finite(i64 n, const double* __restrict__ x, unsigned* out) {
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n && !isfinite(x[idx])) atomicOr(out + 2, 1u);
}

// Block-wide max, then one atomic per block.
__device__ __forceinline__ void block_atomic_max(float x, unsigned* dst) {
  __shared__ float red[16];
  x = wave_max(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) m = fmaxf(m, red[i]);
    if (m > 0.f) atomicMax(dst, __float_as_uint(m));
  }
}

// ---------------------------------------------------------------------------
// Matrix exponential E = exp(alpha H) of one N x N complex matrix (N <= 128),
// one workgroup of 1024 threads.  Scaling and squaring with a Taylor polynomial
// (Moler & Van Loan, "Nineteen dubious ways to compute the exponential of a
// matrix", method 3): X = alpha H / 2^s with ||X||_1 <= 1/2, E = sum_{j<=16}
// X^j / j! by Horner's rule, then s squarings.  Truncation error of the series
// is below ||X||^17 / 17! < 1e-20.  Matrices live in global scratch (L2
// resident); each product stages 16-wide K slabs of both factors in LDS.
// ---------------------------------------------------------------------------
constexpr int EXPM_THREADS = 1024;
constexpr int EXPM_MAXN = 128;

// C = scale A B (+ I if add_eye) (+ C if accumulate); all N x N row-major complex.
__device__ void wg_matmul(int N, const cplx* __restrict__ A, const cplx* __restrict__ B, cplx* C,
                          double scale, bool add_eye, bool accumulate = false) {
  __shared__ cplx sa[EXPM_MAXN][17];
  __shared__ cplx sb[16][EXPM_MAXN + 1];
  const int t = threadIdx.x;
  const int ti = t >> 5, tj = t & 31;        // rows ti + 32a, cols tj + 32b
  cplx acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = mk(0, 0);
  for (int k0 = 0; k0 < N; k0 += 16) {
    __syncthreads();
    for (int e = t; e < EXPM_MAXN * 16; e += EXPM_THREADS) {
      const int r = e >> 4, c = e & 15;
      sa[r][c] = (r < N && k0 + c < N) ? A[r * N + k0 + c] : mk(0, 0);
      const int rb = e / EXPM_MAXN, cb = e % EXPM_MAXN;
      sb[rb][cb] = (k0 + rb < N && cb < N) ? B[(k0 + rb) * N + cb] : mk(0, 0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      cplx av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sa[ti + 32 * a][kk];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sb[kk][tj + 32 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b][0] = fma(av[a][0], bv[b][0], fma(-av[a][1], bv[b][1], acc[a][b][0]));
          acc[a][b][1] = fma(av[a][0], bv[b][1], fma(av[a][1], bv[b][0], acc[a][b][1]));
        }
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ti + 32 * a, j = tj + 32 * b;
      if (i < N && j < N) {
        cplx r = acc[a][b] * scale;
        if (add_eye && i == j) r[0] += 1.0;
        if (accumulate) r += C[i * N + j];
        C[i * N + j] = r;
      }
    }
  __syncthreads();
}

// E = exp(alpha H); scratch: 2 N^2 complex.
__global__ void __launch_bounds__(EXPM_THREADS)
k_expm(int N, const cplx* __restrict__ H, double alpha_re, double alpha_im, cplx* __restrict__ E,
       cplx* __restrict__ X, cplx* __restrict__ S) {
  __shared__ double colsum[EXPM_MAXN];
  __shared__ int s_sh;
  const int t = threadIdx.x;
  const cplx alpha = mk(alpha_re, alpha_im);
  for (int e = t; e < N * N; e += EXPM_THREADS) X[e] = cmul(alpha, H[e]);
  __syncthreads();
  // ||X||_1 = max_j sum_i |X_ij|
  for (int j = t; j < N; j += EXPM_THREADS) {
    double s = 0;
    for (int i = 0; i < N; ++i) {
      const cplx x = X[i * N + j];
      s += sqrt(x[0] * x[0] + x[1] * x[1]);
    }
    colsum[j] = s;
  }
  __syncthreads();
  if (t == 0) {
    double nrm = 0;
    for (int j = 0; j < N; ++j) nrm = fmax(nrm, colsum[j]);
    int s = 0;
    while (nrm > 0.5 && s < 1000) { nrm *= 0.5; ++s; }
    s_sh = s;
  }
  __syncthreads();
  const int s = s_sh;
  const double sc = ldexp(1.0, -s);
  for (int e = t; e < N * N; e += EXPM_THREADS) {
    X[e] = X[e] * sc;
    const int i = e / N, j = e - (e / N) * N;
    E[e] = mk(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // Horner: E <- I + X E / j, j = 16..1
  for (int j = 16; j >= 1; --j) {
    wg_matmul(N, X, E, S, 1.0 / j, true);
    for (int e = t; e < N * N; e += EXPM_THREADS) E[e] = S[e];
    __syncthreads();
  }
  for (int q = 0; q < s; ++q) {
    wg_matmul(N, E, E, S, 1.0, false);
    for (int e = t; e < N * N; e += EXPM_THREADS) E[e] = S[e];
    __syncthreads();
  }
}

// Frechet derivative of the exponential: Lout = L_exp(B, D) with
// B = alpha op(H), op(H) = H or H^dag.  The pair (exp(X), L_exp(X, F)) is
// carried through the same scaling, Taylor (Horner) and squaring steps as
// k_expm: Horner on E <- I + X E / j gives L <- (F E + X L) / j, and a
// squaring E <- E E gives L <- E L + L E (Higham, "Functions of Matrices",
// Sec. 10.6; Al-Mohy & Higham 2009).  Scratch: 6 N^2 complex.
__global__ void __launch_bounds__(EXPM_THREADS)
k_expm_frechet(int N, const cplx* __restrict__ H, int dagger, double alpha_re, double alpha_im,
               const cplx* __restrict__ D, cplx* __restrict__ Lout, cplx* __restrict__ scr) {
  __shared__ double colsum[EXPM_MAXN];
  __shared__ int s_sh;
  const int t = threadIdx.x;
  const int nn = N * N;
  cplx* X = scr;
  cplx* F = scr + nn;
  cplx* E = scr + 2 * nn;
  cplx* L = scr + 3 * nn;
  cplx* T1 = scr + 4 * nn;
  cplx* T2 = scr + 5 * nn;
  const cplx alpha = mk(alpha_re, alpha_im);
  for (int e = t; e < nn; e += EXPM_THREADS) {
    const int i = e / N, j = e - (e / N) * N;
    const cplx hv = dagger ? conj_(H[j * N + i]) : H[e];
    X[e] = cmul(alpha, hv);
  }
  __syncthreads();
  for (int j = t; j < N; j += EXPM_THREADS) {
    double sum = 0;
    for (int i = 0; i < N; ++i) {
      const cplx x = X[i * N + j];
      sum += sqrt(x[0] * x[0] + x[1] * x[1]);
    }
    colsum[j] = sum;
  }
  __syncthreads();
  if (t == 0) {
    double nrm = 0;
    for (int j = 0; j < N; ++j) nrm = fmax(nrm, colsum[j]);
    int sq = 0;
    while (nrm > 0.5 && sq < 1000) { nrm *= 0.5; ++sq; }
    s_sh = sq;
  }
  __syncthreads();
  const int sq = s_sh;
  const double sc = ldexp(1.0, -sq);
  for (int e = t; e < nn; e += EXPM_THREADS) {
    const int i = e / N, j = e - (e / N) * N;
    X[e] = X[e] * sc;
    F[e] = D[e] * sc;
    E[e] = mk(i == j ? 1.0 : 0.0, 0.0);
    L[e] = mk(0.0, 0.0);
  }
  __syncthreads();
  for (int j = 16; j >= 1; --j) {
    wg_matmul(N, F, E, T1, 1.0 / j, false);
    wg_matmul(N, X, L, T1, 1.0 / j, false, true);
    wg_matmul(N, X, E, T2, 1.0 / j, true);
    for (int e = t; e < nn; e += EXPM_THREADS) {
      L[e] = T1[e];
      E[e] = T2[e];
    }
    __syncthreads();
  }
  for (int q = 0; q < sq; ++q) {
    wg_matmul(N, E, L, T1, 1.0, false);
    wg_matmul(N, L, E, T1, 1.0, false, true);
    wg_matmul(N, E, E, T2, 1.0, false);
    for (int e = t; e < nn; e += EXPM_THREADS) {
      L[e] = T1[e];
      E[e] = T2[e];
    }
    __syncthreads();
  }
  for (int e = t; e < nn; e += EXPM_THREADS) Lout[e] = L[e];
}

// ---------------------------------------------------------------------------
// GKBA two-time slices from U_k, X_k = U_k rho_k and Y_k = rho_k U_k^dag:
//   G^<(t,t_k) = i X_k,  G^>(t,t_k) = -i (U_k - X_k),
//   G^<(t_k,t) = i Y_k,  G^>(t_k,t) = -i (U_k^dag - Y_k).
// ---------------------------------------------------------------------------
__global__ void k_gkba(int N, int T, const cplx* __restrict__ U, const cplx* __restrict__ X,
                       const cplx* __restrict__ Y, cplx* __restrict__ Gl, cplx* __restrict__ Gg,
                       cplx* __restrict__ Glb, cplx* __restrict__ Ggb) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const i64 nn = (i64)N * N;
  if (e >= nn * T) return;
  const i64 k = e / nn;
  const int r = (int)(e - k * nn);
  const int i = r / N, j = r - (r / N) * N;
  const cplx u = U[e], x = X[e], y = Y[e];
  const cplx ud = conj_(U[k * nn + (i64)j * N + i]);
  Gl[e] = times_i(x);
  Gg[e] = times_mi(u - x);
  Glb[e] = times_i(y);
  Ggb[e] = times_mi(ud - y);
}

// ---------------------------------------------------------------------------
// Per-chunk operand packing.  Slice b = 2 (k - k0) + sigma holds
//   sigma = 0:  G = G^<(t,t_k), Gbar = G^>(t_k,t)   (-> Sigma^<)
//   sigma = 1:  G = G^>(t,t_k), Gbar = G^<(t_k,t)   (-> Sigma^>)
// cast to the bulk type T; G is stored as G[b][n][m], Gbar transposed as
// GbT[b][r][s] = Gbar_sr (both K-contiguous for the contraction kernels).
// When gbar_from_g is set, Gbar is formed as -G'^dag from the opposite-kind
// input (per-pair inputs of the self-energy entry point).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_pack(int N, int npairs, const cplx* __restrict__ Gl, const cplx* __restrict__ Gg,
                       const cplx* __restrict__ Glb, const cplx* __restrict__ Ggb, int gbar_from_g,
                       T* __restrict__ Gs, T* __restrict__ GbT, unsigned* gmax, unsigned* gbmax) {
  const i64 nn = (i64)N * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  float mg = 0.f, mb = 0.f;
  if (e < 2 * nn * npairs) {
    const i64 b = e / nn;
    const int r = (int)(e - b * nn);
    const int i = r / N, j = r - (r / N) * N;
    const i64 kp = b >> 1;
    const int sig = (int)(b & 1);
    const cplx gv = sig == 0 ? Gl[kp * nn + r] : Gg[kp * nn + r];
    // Gbar element (j, i) goes to GbT[b][i][j]
    cplx gb;
    if (gbar_from_g) {
      const cplx o = sig == 0 ? Gg[kp * nn + r] : Gl[kp * nn + r];   // Gbar_ji = -conj(o_ij)
      gb = mk(-o[0], o[1]);
    } else {
      gb = sig == 0 ? Ggb[kp * nn + (i64)j * N + i] : Glb[kp * nn + (i64)j * N + i];
    }
    Gs[2 * e] = (T)gv[0];
    Gs[2 * e + 1] = (T)gv[1];
    GbT[2 * e] = (T)gb[0];
    GbT[2 * e + 1] = (T)gb[1];
    mg = fmaxf(fabsf((float)gv[0]), fabsf((float)gv[1]));
    mb = fmaxf(fabsf((float)gb[0]), fabsf((float)gb[1]));
  }
  if (gmax) {
    block_atomic_max(mg, gmax);
    __syncthreads();
    block_atomic_max(mb, gbmax);
  }
}

// Element v_abcd of the interaction tensor as the layout kernels read it:
// dense row-major (v[((a N + b) N + c) N + d]) or 8-fold packed (Eq. 4: one
// value per unordered pair of the unordered pairs {a, d} and {b, c},
// packed[tri(tri(a, d), tri(b, c))] with tri(x, y) = max (max + 1) / 2 + min).
// ---------------------------------------------------------------------------
__device__ __forceinline__ i64 v8_tri(i64 a, i64 b) {
  const i64 hi = a > b ? a : b, lo = a > b ? b : a;
  return hi * (hi + 1) / 2 + lo;
}
template <bool PACKED>
__device__ __forceinline__ double v_at(const double* __restrict__ v, int N, int a, int b, int c, int d) {
  if constexpr (PACKED) return v[v8_tri(v8_tri(a, d), v8_tri(b, c))];
  else return v[(((i64)a * N + b) * N + c) * N + d];
}

// ---------------------------------------------------------------------------
// Interaction layouts for the contraction chain:
//   W_T[x][m], x = (j N + s) N + q:  w_mqsj = 2 v_mqsj - v_qmsj   (row pitch KpW)
//   V'[i][n nstride + p N + r] = v_irpn  (row pitch KpV; nstride = N^2, or N^2
//                                         rounded up to 8 for the n-chunked layout)
// Stored in the bulk type, or (split float16) as hi / lo planes of
// x 2^e with 2^e from the recorded max (two passes: k_max_vw, then the writers).
// ---------------------------------------------------------------------------
template <bool PACKED>
__global__ void __launch_bounds__(256) k_max_vw(int N, const double* __restrict__ v, unsigned* vmax,
                                                 unsigned* wmax) {
  const int m = blockIdx.x / N, q = blockIdx.x % N;
  const int nn = N * N;
  float mv = 0.f, mw = 0.f;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int s = e / N, j = e - (e / N) * N;
    const double a = v_at<PACKED>(v, N, m, q, s, j), b = v_at<PACKED>(v, N, q, m, s, j);
    mv = fmaxf(mv, fabsf((float)a));
    mw = fmaxf(mw, fabsf((float)(2.0 * a - b)));
  }
  block_atomic_max(mv, vmax);
  __syncthreads();
  block_atomic_max(mw, wmax);
}

template <typename T>
__device__ __forceinline__ void put_val(T* base, i64 plane, i64 idx, double x, float sc) {
  base[idx] = (T)x;
}
template <>
__device__ __forceinline__ void put_val<_Float16>(_Float16* base, i64 plane, i64 idx, double x, float sc) {
  const float y = (float)x * sc;
  const _Float16 hi = (_Float16)y;
  base[idx] = hi;
  base[plane + idx] = (_Float16)(y - (float)hi);
}

// one workgroup per (s, j-block of 16, m-block of 8); LDS tile [q][j][m]
template <typename T, bool PACKED>
__global__ void __launch_bounds__(256) k_prep_wt(int N, int KpW, const double* __restrict__ v, T* __restrict__ W,
                                                  i64 plane, const unsigned* wmax) {
  __shared__ float tile[128][16][9];
  const int nj = (N + 15) / 16, nm = (N + 7) / 8;
  const int s = blockIdx.x / (nj * nm);
  const int rem = blockIdx.x - s * nj * nm;
  const int j0 = (rem / nm) * 16, m0 = (rem % nm) * 8;
  const float sc = split_scale(wmax);
  // read: for (mm, q): 16 consecutive j of v[m][q][s][j] and v[q][m][s][j]
  for (int L = threadIdx.x; L < 8 * N * 16; L += blockDim.x) {
    const int jj = L & 15, mq = L >> 4;
    const int mm = mq / N, q = mq - (mq / N) * N;
    const int m = m0 + mm, j = j0 + jj;
    float w = 0.f;
    if (m < N && j < N) {
      const double a = v_at<PACKED>(v, N, m, q, s, j);
      const double b = v_at<PACKED>(v, N, q, m, s, j);
      w = (float)(2.0 * a - b);
      if constexpr (sizeof(T) == 8) w = 0.f;    // float64 path re-reads below in full precision
    }
    tile[q][jj][mm] = w;
  }
  __syncthreads();
  // write rows x = (j, s, q), elements m0..m0+7; the row padding m = N .. KpW-1
  // is written as zeros (readers may load whole 8-element groups)
  for (int L = threadIdx.x; L < 16 * N * 8; L += blockDim.x) {
    const int mm = L & 7, jq = L >> 3;
    const int jj = jq / N, q = jq - (jq / N) * N;
    const int m = m0 + mm, j = j0 + jj;
    if (m < KpW && j < N) {
      const i64 x = ((i64)j * N + s) * N + q;
      double val = 0.0;
      if (m < N) {
        if constexpr (sizeof(T) == 8) {
          val = 2.0 * v_at<PACKED>(v, N, m, q, s, j) - v_at<PACKED>(v, N, q, m, s, j);
        } else {
          val = tile[q][jj][mm];
        }
      }
      put_val<T>(W, plane, x * KpW + m, val, sc);
    }
  }
}

// one workgroup per (i, p): 32 x 32 LDS transposes of the (r, n) block
template <typename T, bool PACKED>
__global__ void __launch_bounds__(256) k_prep_vpt(int N, i64 KpV, i64 nstride, const double* __restrict__ v,
                                                   T* __restrict__ Vp, i64 plane, const unsigned* vmax) {
  __shared__ double tile[32][33];
  const int i = blockIdx.x / N, p = blockIdx.x % N;
  const float sc = split_scale(vmax);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r0 = 0; r0 < N; r0 += 32)
    for (int n0 = 0; n0 < N; n0 += 32) {
      __syncthreads();
      for (int yy = ty; yy < 32; yy += 8) {
        const int r = r0 + yy, n = n0 + tx;
        tile[yy][tx] = (r < N && n < N) ? v_at<PACKED>(v, N, i, r, p, n) : 0.0;
      }
      __syncthreads();
      for (int yy = ty; yy < 32; yy += 8) {
        const int n = n0 + yy, r = r0 + tx;
        if (r < N && n < N) put_val<T>(Vp, plane, (i64)i * KpV + (i64)n * nstride + (i64)p * N + r, tile[tx][yy], sc);
      }
    }
}

// ---------------------------------------------------------------------------
// Split-K reduction of the last contraction: part[z][i][c], c = b N + j over
// the chunk's slices, summed over z in order (float64) into
//   S_less[k][i][j] (b even) / S_great[k][i][j] (b odd), k = k0 + b/2,
// and optionally copied into a second destination of the same layout.
// ---------------------------------------------------------------------------
__global__ void k_reduce_sigma(int N, int nslices, int nz, const cplx* __restrict__ part, i64 kbase,
                               cplx* __restrict__ S_less, cplx* __restrict__ S_great,
                               cplx* __restrict__ O_less, cplx* __restrict__ O_great) {
  const i64 ncol = (i64)nslices * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncol * N) return;
  const int i = (int)(e / ncol);
  const i64 c = e - (i64)i * ncol;
  const i64 b = c / N;
  const int j = (int)(c - b * N);
  cplx acc = mk(0, 0);
  for (int z = 0; z < nz; ++z) acc += part[(i64)z * N * ncol + e];
  const i64 k = kbase + (b >> 1);
  const i64 o = k * N * N + (i64)i * N + j;
  if (b & 1) {
    S_great[o] = acc;
    if (O_great) O_great[o] = acc;
  } else {
    S_less[o] = acc;
    if (O_less) O_less[o] = acc;
  }
}

// I = dt sum_k terms[k], the k-sum in k order in float64.
// I = dt sum_k terms_k, k in order; with a time-dependent coupling lam (lam[k]
// = lambda(t_k), the self-energy Sigma(t, t_k) carrying lambda(t) lambda(t_k))
// I = dt lam[now] sum_k lam[k] terms_k.
__global__ void k_sum_terms(int N, int T, const cplx* __restrict__ terms, double dt, cplx* __restrict__ I,
                            const double* __restrict__ lam, int now) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const i64 nn = (i64)N * N;
  if (e >= nn) return;
  cplx acc = mk(0, 0);
  if (lam) {
    for (int k = 0; k < T; ++k) acc += lam[k] * terms[k * nn + e];
    I[e] = acc * (dt * lam[now]);
  } else {
    for (int k = 0; k < T; ++k) acc += terms[k * nn + e];
    I[e] = acc * dt;
  }
}

// rho_out = Y - dt (I + I^dag)
__global__ void k_rho_finish(int N, const cplx* __restrict__ Y, const cplx* __restrict__ I, double dt,
                             cplx* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int i = e / N, j = e - (e / N) * N;
  const cplx a = I[e], b = conj_(I[j * N + i]);
  out[e] = Y[e] - (a + b) * dt;
}

// Effective one-body matrix out = h + Sigma_HF(rho) (with_hf = 0: out = h),
// Eq. 12: (Sigma_HF)_ij = sum_kl (2 v_iklj - v_ikjl) rho_lk, float64.
// Workgroup i (N <= SIGMA_HF_THREADS), thread j; for every k the column
// rho[:, k] is staged in LDS and the (i, k) slab v[i][k][:][:] is read once
// per term: v_iklj along the row l (coalesced over j), v_ikjl along row j.
constexpr int SIGMA_HF_THREADS = 128;
__global__ void __launch_bounds__(SIGMA_HF_THREADS)
k_sigma_hf(int N, const double* __restrict__ v, const cplx* __restrict__ rho, const cplx* __restrict__ h,
           int with_hf, cplx* __restrict__ out, const double* __restrict__ lam, int now) {
  __shared__ cplx col[SIGMA_HF_THREADS];
  const int i = blockIdx.x, j = threadIdx.x;
  const i64 nn = (i64)N * N;
  cplx acc = mk(0.0, 0.0);
  if (with_hf) {
    for (int k = 0; k < N; ++k) {
      __syncthreads();
      if (j < N) col[j] = rho[(i64)j * N + k];
      __syncthreads();
      if (j < N) {
        const double* slab = v + ((i64)i * N + k) * nn;   // slab[l][m] = v[i][k][l][m]
        const double* row = slab + (i64)j * N;            // v_ikjl over l
        for (int l = 0; l < N; ++l) acc += col[l] * (2.0 * slab[(i64)l * N + j] - row[l]);
      }
    }
  }
  if (lam) acc *= lam[now];                               // coupling lambda(t_now)
  if (j < N) out[(i64)i * N + j] = h[(i64)i * N + j] + acc;
}

// h + Sigma_HF (Eq. 12) for the special vertices of Sec. III, written out:
//   diagonal basis  (v_ijkl = U_i d_ij d_ik d_il): Sigma_HF = diag(U_i rho_ii)
//   symmetric basis (v_ijkl = V_ij d_il d_jk):     Sigma_HF_ij = 2 d_ij sum_k V_ik rho_kk - V_ij rho_ij
// p: U (N) or V (N x N, row-major).  One thread per element (i, j).
__global__ void k_sigma_hf_vertex(int N, int symmetric, const double* __restrict__ p, const cplx* __restrict__ rho,
                                  const cplx* __restrict__ h, int with_hf, cplx* __restrict__ out) {
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (i64)N * N) return;
  const int i = (int)(idx / N), j = (int)(idx - (i64)i * N);
  cplx acc = h[idx];
  if (with_hf) {
    if (!symmetric) {
      if (i == j) acc += p[i] * rho[idx];
    } else {
      if (i == j)
        for (int k = 0; k < N; ++k) acc += 2.0 * p[(i64)i * N + k] * rho[(i64)k * N + k];
      acc -= p[idx] * rho[idx];
    }
  }
  out[idx] = acc;
}

// ---------------------------------------------------------------------------
// Self-energy of the special vertices (Sec. III A, III B), float64, for T
// slices of one kind: G[k] = G(t, t_k) and Gb[k] = Gbar (the opposite-kind
// function at (t_k, t)), row-major N x N each.
// ---------------------------------------------------------------------------

// Diagonal basis, Eq. 14: S_ij = U_i U_j G_ij Gb_ji G_ij.
__global__ void k_sigma_diag(int N, int T, const double* __restrict__ u, const cplx* __restrict__ G,
                             const cplx* __restrict__ Gb, cplx* __restrict__ S) {
  const i64 nn = (i64)N * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn * T) return;
  const i64 k = e / nn;
  const int r = (int)(e - k * nn);
  const int i = r / N, j = r - (r / N) * N;
  const cplx g = G[e];
  S[e] = cmul(cmul(g, Gb[k * nn + (i64)j * N + i]), g) * (u[i] * u[j]);
}

// Symmetric basis, bubble operand of Eq. 17: P_ab = Gb_ba G_ab.
__global__ void k_sym_bubble_in(int N, int T, const cplx* __restrict__ G, const cplx* __restrict__ Gb,
                                cplx* __restrict__ P) {
  const i64 nn = (i64)N * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn * T) return;
  const i64 k = e / nn;
  const int r = (int)(e - k * nn);
  const int a = r / N, b = r - (r / N) * N;
  P[e] = cmul(Gb[k * nn + (i64)b * N + a], G[e]);
}

// Symmetric basis, exchange operand: A[k][i][l][m] = G_il Gb_lm V_im, so that
// (A[k][i] x G)_lj summed against V_jl over l gives the exchange term
// sum_{m,l} V_im V_jl G_il Gb_lm G_mj of Eq. 16.
__global__ void k_sym_exch_in(int N, int T, const double* __restrict__ V, const cplx* __restrict__ G,
                              const cplx* __restrict__ Gb, cplx* __restrict__ A) {
  const i64 nn = (i64)N * N, n3 = nn * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3 * T) return;
  const i64 k = e / n3;
  const i64 r = e - k * n3;
  const int i = (int)(r / nn);
  const int lm = (int)(r - (i64)i * nn);
  const int l = lm / N, m = lm - (lm / N) * N;
  A[e] = cmul(G[k * nn + (i64)i * N + l], Gb[k * nn + lm]) * V[(i64)i * N + m];
}

// S_ij = 2 G_ij R_ji - sum_l V_jl B[k][i]_lj  (bubble R = V (V P)^T, Eq. 17;
// exchange from B[k][i] = A[k][i] x G, Eq. 16).
__global__ void k_sym_finish(int N, int T, const double* __restrict__ V, const cplx* __restrict__ G,
                             const cplx* __restrict__ R, const cplx* __restrict__ B, cplx* __restrict__ S) {
  const i64 nn = (i64)N * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn * T) return;
  const i64 k = e / nn;
  const int r = (int)(e - k * nn);
  const int i = r / N, j = r - (r / N) * N;
  const cplx* b = B + (k * N + i) * nn + j;
  cplx x = mk(0.0, 0.0);
  for (int l = 0; l < N; ++l) x += b[(i64)l * N] * V[(i64)j * N + l];
  S[e] = cmul(G[e], R[k * nn + (i64)j * N + i]) * 2.0 - x;
}

// y = x + 0 i
__global__ void k_real_to_c(i64 n, const double* __restrict__ x, cplx* __restrict__ y) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = mk(x[e], 0.0);
}

// ---------------------------------------------------------------------------
// 8-fold packed interaction tensor (real orbitals, Eq. 4): v_ijkl depends only
// on the unordered pairs {i, l} (the orbitals at r) and {j, k} (at r') and on
// their order, so it is stored once per unordered pair of unordered pairs:
//   pair(a, b) = max(a,b) (max(a,b) + 1) / 2 + min(a,b),
//   packed[ tri(P, Q) ],  P = pair(i, l), Q = pair(j, k),
//   tri(P, Q) = max(P,Q) (max(P,Q) + 1) / 2 + min(P,Q).
// ---------------------------------------------------------------------------
// v[i][j][k][l] = packed[tri(pair(i, l), pair(j, k))] for all N^4 entries.
__global__ void k_v8_expand(int N, const double* __restrict__ packed, double* __restrict__ v) {
  const i64 nn = (i64)N * N, total = nn * nn;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const i64 ij = e / nn, kl = e - ij * nn;         // e = (i N + j) N^2 + (k N + l)
  const int i = (int)(ij / N), j = (int)(ij - (ij / N) * N);
  const int k = (int)(kl / N), l = (int)(kl - (kl / N) * N);
  v[e] = packed[v8_tri(v8_tri(i, l), v8_tri(j, k))];
}

// x <- (a + i b) x
__global__ void k_scale_c(i64 n, cplx* __restrict__ x, double a, double b) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = cmul(mk(a, b), x[e]);
}

// x <- lam[idx] x for n complex values (a coupling weight read on the device)
__global__ void k_scale_by(i64 n, cplx* __restrict__ x, const double* __restrict__ lam, int idx) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = x[e] * lam[idx];
}

// out <- the N x N identity
__global__ void k_eye_c(int N, cplx* __restrict__ out) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (i64)N * N) out[e] = mk(e % (N + 1) == 0 ? 1.0 : 0.0, 0.0);
}

// out <- in^dag (N x N complex)
__global__ void k_adjoint_c(int N, const cplx* __restrict__ in, cplx* __restrict__ out) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (i64)N * N) return;
  const int i = (int)(e / N), j = (int)(e - (e / N) * N);
  out[e] = conj_(in[(i64)j * N + i]);
}

// out <- a + b (complex)
__global__ void k_add_c(i64 n, const cplx* __restrict__ a, const cplx* __restrict__ b, cplx* __restrict__ out) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = a[e] + b[e];
}

// Strided complex copy, used to lay out small operands.
__global__ void k_copy(i64 n, const cplx* __restrict__ src, cplx* __restrict__ dst) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

// ---------------------------------------------------------------------------
// Adjoint helpers (float64)
// ---------------------------------------------------------------------------

// out[e] (+)= sum_z part[z count + e]
__global__ void k_sum_partials(i64 count, int nz, const cplx* __restrict__ part, cplx* __restrict__ out,
                               int accumulate) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  cplx acc = accumulate ? out[e] : mk(0, 0);
  for (int z = 0; z < nz; ++z) acc += part[(i64)z * count + e];
  out[e] = acc;
}

// slice cotangents of a chunk: gSs[b] = dL/dSigma of slice b, gSt[i][b][j] = gSs[b][i][j]
__global__ void k_pack_gs(int N, int npairs, const cplx* __restrict__ gSl, const cplx* __restrict__ gSg,
                          cplx* __restrict__ gSs, cplx* __restrict__ gSt) {
  const i64 nn = (i64)N * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * nn * npairs) return;
  const i64 b = e / nn;
  const int r = (int)(e - b * nn);
  const int i = r / N, j = r - (r / N) * N;
  const i64 kp = b >> 1;
  const cplx x = (b & 1) ? gSg[kp * nn + r] : gSl[kp * nn + r];
  gSs[e] = x;
  gSt[(i64)i * (2 * npairs) * N + b * N + j] = x;
}

// chain cotangents of the slices back onto the GKBA functions of the chunk
__global__ void k_scatter_gg(int N, int npairs, const cplx* __restrict__ gGs, const cplx* __restrict__ gGbs,
                             cplx* __restrict__ gGl, cplx* __restrict__ gGg, cplx* __restrict__ gGlb,
                             cplx* __restrict__ gGgb) {
  const i64 nn = (i64)N * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn * npairs) return;
  const i64 kp = e / nn;
  const i64 r = e - kp * nn;
  gGl[e] = gGs[(2 * kp) * nn + r];
  gGg[e] = gGs[(2 * kp + 1) * nn + r];
  gGgb[e] += gGbs[(2 * kp) * nn + r];
  gGlb[e] += gGbs[(2 * kp + 1) * nn + r];
}

// GKBA adjoint, elementwise part:
//   gX = -i (gGl + gGg),  gY = -i (gGlb + gGgb),  gU = i gGg - i gGgb^dag
__global__ void k_gkba_adj(int N, int T, const cplx* __restrict__ gGl, const cplx* __restrict__ gGg,
                           const cplx* __restrict__ gGlb, const cplx* __restrict__ gGgb, cplx* __restrict__ gX,
                           cplx* __restrict__ gY, cplx* __restrict__ gU) {
  const i64 nn = (i64)N * N;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn * T) return;
  const i64 k = e / nn;
  const int r = (int)(e - k * nn);
  const int i = r / N, j = r - (r / N) * N;
  gX[e] = times_mi(gGl[e] + gGg[e]);
  gY[e] = times_mi(gGlb[e] + gGgb[e]);
  const cplx gd = conj_(gGgb[k * nn + (i64)j * N + i]);
  gU[e] = times_i(gGg[e]) - times_i(gd);
}

// gv_ijkl = 2 gw_ijkl - gw_jikl + gVp[i][(l,k,j)],  gw_mqsj = gWT[(j,s,q)][m]
__global__ void k_assemble_gv(int N, const double* __restrict__ gWT, const double* __restrict__ gVp,
                              double* __restrict__ gv) {
  const i64 n = N, n3 = n * n * n;
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3 * n) return;
  const int l = (int)(e % n), k = (int)((e / n) % n), j = (int)((e / (n * n)) % n), i = (int)(e / n3);
  const i64 lk = ((i64)l * N + k) * N;
  gv[e] = 2.0 * gWT[(lk + j) * N + i] - gWT[(lk + i) * N + j] + gVp[(i64)i * n3 + lk + j];
}

}  // namespace sb2
