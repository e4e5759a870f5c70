// Batched, strided complex GEMM on the CDNA4 matrix cores (gfx950).
//
//   C[z](m, n) (+)= alpha * sum_k opA(A[z])(m, k) * opB(B[z])(k, n)
//
// for complex or real operands, with per-operand element strides, a two-level
// batch index, a two-level output row index and split-K.  Every contraction of
// the second-Born chain, of the GKBA set-up and of the adjoint is one launch of
// this kernel with suitable strides.
//
// Work decomposition: a workgroup of WM x WN wave64s owns a BM x BN output tile
// (BM = 16 FM WM, BN = 16 FN WN); each wave owns FM x FN 16x16 MFMA fragments
// and keeps a real and an imaginary accumulator per fragment.  K is walked in
// BK-deep slabs staged through LDS with a register prefetch of the next slab
// (two LDS buffers, one barrier per slab).  A complex x complex product costs
// four real MFMAs (no 3-multiply trick, so no extra cancellation).
//
// Precisions:
//   * double: v_mfma_f64_16x16x4_f64, float64 accumulation.
//   * float : v_mfma_f32_16x16x4_f32, float32 accumulation; with ACC64 the
//             float32 partial is folded into a float64 accumulator every
//             `kpromote` slabs, which bounds the float32 summation length along
//             very long contractions.
//   * split float16 (k_gemm_h16): operands are stored as float32; at LDS-store
//             time each value x is scaled by a power of two 2^e (chosen from the
//             operand's recorded max |x| so that |x 2^e| < 2^14) and split into
//             hi = fp16(x 2^e), lo = fp16(x 2^e - hi).  A real product uses
//             three v_mfma_f32_16x16x32_f16: hi*hi + hi*lo + lo*hi, accumulated
//             in float32; the epilogue removes the scales exactly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sb2 {

typedef long long i64;
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));
typedef _Float16 hx8 __attribute__((ext_vector_type(8)));
typedef unsigned ux4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
  int M, N, K;
  int nbl;                 // batch index z = bh * nbl + bl
  int kchunk;              // split-K: blockIdx.z covers k in [z kchunk, min(K, (z+1) kchunk))
  int tiles_m;             // row tiles; blockIdx.x = tm + tiles_m * tn
  const void* A; i64 sAm, sAk, sAbh, sAbl;
  const void* B; i64 sBk, sBn, sBbh, sBbl;
  void* C; i64 sCm, sCn, sCbh, sCbl, sCz;
  int Mlo; i64 sCmh;       // Mlo > 0: m = mh Mlo + ml addresses mh sCmh + ml sCm
  int Klo; i64 sAkh, sBkh; // K2 kernels: k = kh Klo + kl addresses kh s*kh + kl s*k
  int conjA, conjB;
  double alpha_re, alpha_im;
  int beta1;               // accumulate into C instead of overwriting
  int out_real;            // C is real: store Re(alpha acc) only
  int kpromote;            // ACC64: fold float32 partials every kpromote slabs
  const unsigned* amax;    // split: max |A| as float bits (scale source), may be null
  const unsigned* bmax;    // split: max |B| as float bits, may be null
  unsigned* cmax;          // split producer: atomically raised to max |C| written, may be null
};

// ---------------------------------------------------------------------------
// MFMA wrappers.  Inputs (16x16xK): lane l supplies A[l%16][k] and B[k][l%16]
// for k = l/16 (K = 4) or k = 8(l/16)..8(l/16)+7 (K = 32).  Output fragment:
// lane l holds column l%16 and, in accumulator slot q, row
//   f32 / f16 instructions:  4 (l/16) + q
//   f64 instruction:         (l/16) + 4 q
// (checked with a lane-layout probe on gfx950).
// ---------------------------------------------------------------------------
template <typename T> struct Acc;
template <> struct Acc<double> { using type = dx4; };
template <> struct Acc<float> { using type = fx4; };

// row of accumulator slot q held by lane group kq = l/16
template <typename T> __device__ __forceinline__ int frag_row(int kq, int q);
template <> __device__ __forceinline__ int frag_row<double>(int kq, int q) { return kq + 4 * q; }
template <> __device__ __forceinline__ int frag_row<float>(int kq, int q) { return 4 * kq + q; }

__device__ __forceinline__ dx4 mma(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mma(float a, float b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mma16(hx8 a, hx8 b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
// hi*hi + hi*lo + lo*hi
__device__ __forceinline__ fx4 mma3(hx8 ah, hx8 al, hx8 bh, hx8 bl, fx4 c) {
  c = mma16(al, bh, c);
  c = mma16(ah, bl, c);
  return mma16(ah, bh, c);
}

// Split of two scaled values x0 s0, x1 s1 into packed float16 pairs
// h = [f16(x0 s0), f16(x1 s1)] and l = [f16(x0 s0 - h0), f16(x1 s1 - h1)].
// Each half is one mixed-precision fused multiply-add that rounds once to
// float16 (the low-part one takes its h operand as a float16 half of h), so a
// pair costs four instructions.  With s a power of two or zero, x s is exact
// in float32 and the halves equal f16(x s) and f16(x s - f16(x s)).
// The compiler does not insert matrix-core wait states around inline
// assembly: the inputs must not be fresh MFMA results and the outputs must not
// feed an MFMA directly (here they come from memory loads and go to LDS).
__device__ __forceinline__ void split_pair(float x0, float s0, float x1, float s1, unsigned& h, unsigned& l) {
  asm("v_fma_mixlo_f16 %0, %2, %3, 0\n\t"
      "v_fma_mixhi_f16 %0, %4, %5, 0\n\t"
      "v_fma_mixlo_f16 %1, %2, %3, -%0 op_sel_hi:[0,0,1]\n\t"
      "v_fma_mixhi_f16 %1, %4, %5, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
      : "=&v"(h), "=&v"(l)
      : "v"(x0), "v"(s0), "v"(x1), "v"(s1));
}

template <typename V> __device__ __forceinline__ V vzero() {
  V v;
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = 0;
  return v;
}

// ---------------------------------------------------------------------------
// Global tile loader: R x Cc tile, element (r, c) at base + r sr + c sc (in
// elements; a complex element is two scalars).  Element e of thread t is linear
// index L = t + e NT, walked with c fastest when cfast (sc == 1), else r fastest,
// so that consecutive lanes read consecutive addresses.
// ---------------------------------------------------------------------------
template <typename T, bool CPLX, int R, int Cc, int NT>
struct TileRegs {
  static constexpr int E = (R * Cc + NT - 1) / NT;
  T re[E];
  T im[E];

  __device__ __forceinline__ static void rc(int L, bool cfast, int& r, int& c) {
    if (cfast) { r = L / Cc; c = L - r * Cc; }
    else { c = L / R; r = L - c * R; }
  }

  template <class Off>
  __device__ __forceinline__ void load(const T* __restrict__ base, Off off_of, int rlim, int clim, bool cfast,
                                       int tid) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int L = tid + e * NT;
      int r, c;
      rc(L, cfast, r, c);
      const bool ok = (L < R * Cc) && r < rlim && c < clim;
      if (ok) {
        const i64 off = off_of(r, c);
        if constexpr (CPLX) {
          typedef T t2 __attribute__((ext_vector_type(2)));
          const t2 x = *reinterpret_cast<const t2*>(base + 2 * off);
          re[e] = x[0];
          im[e] = x[1];
        } else {
          re[e] = base[off];
        }
      } else {
        re[e] = T(0);
        if constexpr (CPLX) im[e] = T(0);
      }
    }
  }

  __device__ __forceinline__ void load(const T* __restrict__ base, i64 sr, i64 sc, int rlim, int clim,
                                       bool cfast, int tid) {
    load(base, [&](int r, int c) { return (i64)r * sr + (i64)c * sc; }, rlim, clim, cfast, tid);
  }
};

template <typename V>
__device__ __forceinline__ float max_abs4(V a) {
  float m = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) m = fmaxf(m, fabsf((float)a[i]));
  return m;
}

// Power-of-two scale that maps max |x| below 2^14 (float16 keeps headroom for lo).
__device__ __forceinline__ float split_scale(const unsigned* mx) {
  if (!mx) return 1.f;
  const float m = __uint_as_float(*mx);
  if (!(m > 0.f) || !(m < 3.0e38f)) return 1.f;
  int e;
  frexpf(m, &e);               // m < 2^e
  return ldexpf(1.f, 14 - e);
}

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

// Output element address offset (in elements).
__device__ __forceinline__ i64 out_off(const GemmArgs& g, int m, int n) {
  i64 om;
  if (g.Mlo > 0) {
    const int mh = m / g.Mlo;
    om = (i64)mh * g.sCmh + (i64)(m - mh * g.Mlo) * g.sCm;
  } else {
    om = (i64)m * g.sCm;
  }
  return om + (i64)n * g.sCn;
}

template <typename OutT>
__device__ __forceinline__ void store_elem(const GemmArgs& g, OutT* Cb, int m, int n, double re, double im) {
  const double ore = g.alpha_re * re - g.alpha_im * im;
  const double oim = g.alpha_re * im + g.alpha_im * re;
  const i64 off = out_off(g, m, n);
  if (g.out_real) {
    OutT* p = Cb + off;
    if (g.beta1) *p = (OutT)((double)*p + ore);
    else *p = (OutT)ore;
  } else {
    OutT* p = Cb + 2 * off;
    if (g.beta1) {
      p[0] = (OutT)((double)p[0] + ore);
      p[1] = (OutT)((double)p[1] + oim);
    } else {
      p[0] = (OutT)ore;
      p[1] = (OutT)oim;
    }
  }
}

// ---------------------------------------------------------------------------
// float64 / float32 kernel
// ---------------------------------------------------------------------------
template <typename T, typename OutT, int WM, int WN, int FM, int FN, bool AC, bool BC, bool ACC64, bool K2 = false>
__global__ void __launch_bounds__(64 * WM * WN)
k_gemm(const GemmArgs g) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = 16 * FM * WM, BN = 16 * FN * WN, BK = 16;
  constexpr int LDA = BM + ((BM % 32) == 0 ? 16 : 0);
  constexpr int LDB = BN + ((BN % 32) == 0 ? 16 : 0);
  constexpr int PA = AC ? 2 : 1, PB = BC ? 2 : 1;
  using acc_t = typename Acc<T>::type;

  __shared__ T sA[2][PA][BK][LDA];
  __shared__ T sB[2][PB][BK][LDB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave - wm * WN;
  const int tm = blockIdx.x % g.tiles_m, tn = blockIdx.x / g.tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int bz = blockIdx.y, bh = bz / g.nbl, bl = bz - bh * g.nbl;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);

  const T* Ab = reinterpret_cast<const T*>(g.A) + PA * ((i64)bh * g.sAbh + (i64)bl * g.sAbl + (i64)m0 * g.sAm);
  const T* Bb = reinterpret_cast<const T*>(g.B) + PB * ((i64)bh * g.sBbh + (i64)bl * g.sBbl + (i64)n0 * g.sBn);
  const int mlim = g.M - m0, nlim = g.N - n0;
  const bool a_cfast = (g.sAk == 1);      // A tile is (m rows) x (k cols)
  const bool b_cfast = (g.sBn == 1);      // B tile is (k rows) x (n cols)
  const T sgnA = g.conjA ? T(-1) : T(1);
  const T sgnB = g.conjB ? T(-1) : T(1);

  TileRegs<T, AC, BM, BK, NT> ra;
  TileRegs<T, BC, BK, BN, NT> rb;

  auto gload = [&](int k0) {
    const int klim = kend - k0;
    if constexpr (K2) {
      // two-level K: element k = kh Klo + kl at kh s*kh + kl s*k.  One division
      // per slab when BK <= Klo: the slab's BK consecutive k cross at most one
      // multiple of Klo, so each element's (kh, kl) is (kh0, kl0 + c) or
      // (kh0 + 1, kl0 + c - Klo).
      if (g.Klo >= BK) {                               // uniform
        const int kh0 = k0 / g.Klo, kl0 = k0 - kh0 * g.Klo;
        const i64 a0 = (i64)kh0 * g.sAkh + (i64)kl0 * g.sAk, b0 = (i64)kh0 * g.sBkh + (i64)kl0 * g.sBk;
        const i64 a_wrap = g.sAkh - (i64)g.Klo * g.sAk, b_wrap = g.sBkh - (i64)g.Klo * g.sBk;
        ra.load(Ab, [&](int r, int c) {
          return (i64)r * g.sAm + a0 + (i64)c * g.sAk + (kl0 + c >= g.Klo ? a_wrap : 0);
        }, mlim, klim, a_cfast, tid);
        rb.load(Bb, [&](int r, int c) {
          return b0 + (i64)r * g.sBk + (kl0 + r >= g.Klo ? b_wrap : 0) + (i64)c * g.sBn;
        }, klim, nlim, b_cfast, tid);
      } else {                                         // Klo < BK (N < 4): a division per element
        ra.load(Ab, [&](int r, int c) {
          const int kk = k0 + c, kh = kk / g.Klo;
          return (i64)r * g.sAm + (i64)kh * g.sAkh + (i64)(kk - kh * g.Klo) * g.sAk;
        }, mlim, klim, a_cfast, tid);
        rb.load(Bb, [&](int r, int c) {
          const int kk = k0 + r, kh = kk / g.Klo;
          return (i64)kh * g.sBkh + (i64)(kk - kh * g.Klo) * g.sBk + (i64)c * g.sBn;
        }, klim, nlim, b_cfast, tid);
      }
    } else {
      ra.load(Ab + PA * (i64)k0 * g.sAk, g.sAm, g.sAk, mlim, klim, a_cfast, tid);
      rb.load(Bb + PB * (i64)k0 * g.sBk, g.sBk, g.sBn, klim, nlim, b_cfast, tid);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < ra.E; ++e) {
      const int L = tid + e * NT;
      if (L < BM * BK) {
        int r, c;
        ra.rc(L, a_cfast, r, c);
        sA[buf][0][c][r] = ra.re[e];
        if constexpr (AC) sA[buf][PA - 1][c][r] = sgnA * ra.im[e];
      }
    }
#pragma unroll
    for (int e = 0; e < rb.E; ++e) {
      const int L = tid + e * NT;
      if (L < BK * BN) {
        int r, c;
        rb.rc(L, b_cfast, r, c);
        sB[buf][0][r][c] = rb.re[e];
        if constexpr (BC) sB[buf][PB - 1][r][c] = sgnB * rb.im[e];
      }
    }
  };

  acc_t cr[FM][FN], ci[FM][FN];
  dx4 dr[ACC64 ? FM : 1][ACC64 ? FN : 1], di[ACC64 ? FM : 1][ACC64 ? FN : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      cr[i][j] = vzero<acc_t>();
      ci[i][j] = vzero<acc_t>();
      if constexpr (ACC64) { dr[i][j] = vzero<dx4>(); di[i][j] = vzero<dx4>(); }
    }

  const int wrow0 = m0 + wm * FM * 16, wcol0 = n0 + wn * FN * 16;

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    lstore(0);
  }
  __syncthreads();
  const int kq = lane >> 4, lr = lane & 15;
  for (int it = 0; it < nk; ++it) {
    const int k0 = kbeg + it * BK;
    const int cur = it & 1;
    if (it + 1 < nk) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      if (k0 + kk * 4 < kend) {
        T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const int row = wm * FM * 16 + i * 16 + lr;
          ar[i] = sA[cur][0][kk * 4 + kq][row];
          if constexpr (AC) ai[i] = sA[cur][PA - 1][kk * 4 + kq][row];
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = wn * FN * 16 + j * 16 + lr;
          br[j] = sB[cur][0][kk * 4 + kq][col];
          if constexpr (BC) bi[j] = sB[cur][PB - 1][kk * 4 + kq][col];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            cr[i][j] = mma(ar[i], br[j], cr[i][j]);
            if constexpr (AC && BC) {
              cr[i][j] = mma(-ai[i], bi[j], cr[i][j]);
              ci[i][j] = mma(ar[i], bi[j], ci[i][j]);
              ci[i][j] = mma(ai[i], br[j], ci[i][j]);
            } else if constexpr (AC) {
              ci[i][j] = mma(ai[i], br[j], ci[i][j]);
            } else if constexpr (BC) {
              ci[i][j] = mma(ar[i], bi[j], ci[i][j]);
            }
          }
        }
      }
    }
    if constexpr (ACC64) {
      if ((it + 1) % g.kpromote == 0 || it + 1 == nk) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              dr[i][j][q] += (double)cr[i][j][q];
              di[i][j][q] += (double)ci[i][j][q];
              cr[i][j][q] = 0;
              ci[i][j][q] = 0;
            }
      }
    }
    if (it + 1 < nk) lstore(cur ^ 1);
    __syncthreads();
  }

  OutT* Cb = reinterpret_cast<OutT*>(g.C);
  const i64 cbase = (i64)bh * g.sCbh + (i64)bl * g.sCbl + (i64)blockIdx.z * g.sCz;
  Cb += (g.out_real ? 1 : 2) * cbase;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = wrow0 + i * 16 + frag_row<T>(kq, q);
        const int n = wcol0 + j * 16 + lr;
        if (m < g.M && n < g.N) {
          double re, im;
          if constexpr (ACC64) { re = dr[i][j][q]; im = di[i][j][q]; }
          else { re = (double)cr[i][j][q]; im = (double)ci[i][j][q]; }
          store_elem<OutT>(g, Cb, m, n, re, im);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// split-float16 kernel (operands stored as float32)
// ---------------------------------------------------------------------------
template <typename OutT, int WM, int WN, int FM, int FN, bool AC, bool BC, bool ACC64>
__global__ void __launch_bounds__(64 * WM * WN)
k_gemm_h16(const GemmArgs g) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = 16 * FM * WM, BN = 16 * FN * WN, BK = 32;
  constexpr int LDK = BK + 8;                  // halves per LDS row (80 bytes)
  constexpr int PA = AC ? 4 : 2, PB = BC ? 4 : 2;  // planes: re_hi, re_lo[, im_hi, im_lo]

  __shared__ __attribute__((aligned(16))) _Float16 sA[2][PA][BM][LDK];
  __shared__ __attribute__((aligned(16))) _Float16 sB[2][PB][BN][LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave - wm * WN;
  const int tm = blockIdx.x % g.tiles_m, tn = blockIdx.x / g.tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int bz = blockIdx.y, bh = bz / g.nbl, bl = bz - bh * g.nbl;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  constexpr int EA = AC ? 2 : 1, EB = BC ? 2 : 1;

  const float* Ab = reinterpret_cast<const float*>(g.A) + EA * ((i64)bh * g.sAbh + (i64)bl * g.sAbl + (i64)m0 * g.sAm);
  const float* Bb = reinterpret_cast<const float*>(g.B) + EB * ((i64)bh * g.sBbh + (i64)bl * g.sBbl + (i64)n0 * g.sBn);
  const int mlim = g.M - m0, nlim = g.N - n0;
  const bool a_cfast = (g.sAk == 1);
  const bool b_cfast = (g.sBn == 1);
  const float scA = split_scale(g.amax), scB = split_scale(g.bmax);
  const float sgnA = g.conjA ? -scA : scA;
  const float sgnB = g.conjB ? -scB : scB;

  TileRegs<float, AC, BM, BK, NT> ra;
  TileRegs<float, BC, BK, BN, NT> rb;

  auto gload = [&](int k0) {
    const int klim = kend - k0;
    ra.load(Ab + EA * (i64)k0 * g.sAk, g.sAm, g.sAk, mlim, klim, a_cfast, tid);
    rb.load(Bb + EB * (i64)k0 * g.sBk, g.sBk, g.sBn, klim, nlim, b_cfast, tid);
  };
  auto split = [](float x, _Float16& hi, _Float16& lo) {
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < ra.E; ++e) {
      const int L = tid + e * NT;
      if (L < BM * BK) {
        int r, c;
        ra.rc(L, a_cfast, r, c);      // r = m, c = k
        split(ra.re[e] * scA, sA[buf][0][r][c], sA[buf][1][r][c]);
        if constexpr (AC) split(ra.im[e] * sgnA, sA[buf][2][r][c], sA[buf][3][r][c]);
      }
    }
#pragma unroll
    for (int e = 0; e < rb.E; ++e) {
      const int L = tid + e * NT;
      if (L < BK * BN) {
        int r, c;
        rb.rc(L, b_cfast, r, c);      // r = k, c = n
        split(rb.re[e] * scB, sB[buf][0][c][r], sB[buf][1][c][r]);
        if constexpr (BC) split(rb.im[e] * sgnB, sB[buf][2][c][r], sB[buf][3][c][r]);
      }
    }
  };

  fx4 cr[FM][FN], ci[FM][FN];
  dx4 dr[ACC64 ? FM : 1][ACC64 ? FN : 1], di[ACC64 ? FM : 1][ACC64 ? FN : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      cr[i][j] = vzero<fx4>();
      ci[i][j] = vzero<fx4>();
      if constexpr (ACC64) { dr[i][j] = vzero<dx4>(); di[i][j] = vzero<dx4>(); }
    }
  const int wrow0 = m0 + wm * FM * 16, wcol0 = n0 + wn * FN * 16;

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    lstore(0);
  }
  __syncthreads();
  const int kq = lane >> 4, lr = lane & 15;
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload(kbeg + (it + 1) * BK);
    hx8 arh[FM], arl[FM], aih[FM], ail[FM], brh[FN], brl[FN], bih[FN], bil[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int row = wm * FM * 16 + i * 16 + lr;
      arh[i] = *reinterpret_cast<const hx8*>(&sA[cur][0][row][8 * kq]);
      arl[i] = *reinterpret_cast<const hx8*>(&sA[cur][1][row][8 * kq]);
      if constexpr (AC) {
        aih[i] = *reinterpret_cast<const hx8*>(&sA[cur][2][row][8 * kq]);
        ail[i] = *reinterpret_cast<const hx8*>(&sA[cur][3][row][8 * kq]);
      }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = wn * FN * 16 + j * 16 + lr;
      brh[j] = *reinterpret_cast<const hx8*>(&sB[cur][0][col][8 * kq]);
      brl[j] = *reinterpret_cast<const hx8*>(&sB[cur][1][col][8 * kq]);
      if constexpr (BC) {
        bih[j] = *reinterpret_cast<const hx8*>(&sB[cur][2][col][8 * kq]);
        bil[j] = *reinterpret_cast<const hx8*>(&sB[cur][3][col][8 * kq]);
      }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = mma3(arh[i], arl[i], brh[j], brl[j], cr[i][j]);
        if constexpr (AC && BC) {
          cr[i][j] = mma3(-aih[i], -ail[i], bih[j], bil[j], cr[i][j]);
          ci[i][j] = mma3(arh[i], arl[i], bih[j], bil[j], ci[i][j]);
          ci[i][j] = mma3(aih[i], ail[i], brh[j], brl[j], ci[i][j]);
        } else if constexpr (AC) {
          ci[i][j] = mma3(aih[i], ail[i], brh[j], brl[j], ci[i][j]);
        } else if constexpr (BC) {
          ci[i][j] = mma3(arh[i], arl[i], bih[j], bil[j], ci[i][j]);
        }
      }
    }
    if constexpr (ACC64) {
      if ((it + 1) % g.kpromote == 0 || it + 1 == nk) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              dr[i][j][q] += (double)cr[i][j][q];
              di[i][j][q] += (double)ci[i][j][q];
              cr[i][j][q] = 0;
              ci[i][j][q] = 0;
            }
      }
    }
    if (it + 1 < nk) lstore(cur ^ 1);
    __syncthreads();
  }

  const double unscale = 1.0 / ((double)scA * (double)scB);
  OutT* Cb = reinterpret_cast<OutT*>(g.C);
  const i64 cbase = (i64)bh * g.sCbh + (i64)bl * g.sCbl + (i64)blockIdx.z * g.sCz;
  Cb += (g.out_real ? 1 : 2) * cbase;
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = wrow0 + i * 16 + frag_row<float>(kq, q);
        const int n = wcol0 + j * 16 + lr;
        if (m < g.M && n < g.N) {
          double re, im;
          if constexpr (ACC64) { re = dr[i][j][q]; im = di[i][j][q]; }
          else { re = (double)cr[i][j][q]; im = (double)ci[i][j][q]; }
          re *= unscale;
          im *= unscale;
          store_elem<OutT>(g, Cb, m, n, re, im);
          const double ore = g.alpha_re * re - g.alpha_im * im;
          const double oim = g.alpha_re * im + g.alpha_im * re;
          mx = fmaxf(mx, fmaxf(fabsf((float)ore), fabsf((float)oim)));
        }
      }
    }
  }
  if (g.cmax) {
    mx = wave_max(mx);
    if (lane == 0 && mx > 0.f) atomicMax(g.cmax, __float_as_uint(mx));
  }
}

}  // namespace sb2
