// Last contraction of the chain for split float16 arithmetic:
//
//   part[n][i][c] = sum_{(p,r)} V'[i][(n,p,r)] C[(b,j)][(n,p,r)],   c = (b, j)
//
// in the n-chunked layout: chunk n of V' is the row segment n KB .. n KB + N^2
// (KB = N^2 rounded up to 8, zero padding), chunk n of C the contiguous block
// [n][c][(p,r)], so one workgroup streams one contiguous region of C.  V'
// (real) arrives pre-split as two float16 planes; C (complex float32) is split
// once, when it is staged.  The N chunks are summed in float64 afterwards;
// within a chunk the float32 MFMA accumulators are folded into float64 once per
// two slabs.
//
// Workgroup: 8 waves = 2 row halves x 4 column groups (two waves per SIMD),
// 64 columns c; wave (h, g) owns the 16 columns 16 g .. 16 g + 15 and the row
// fragments h FH .. h FH + FH - 1 of the FSP >= FS padded fragments.  Slabs of
// 64 k of both operands are staged in LDS, double buffered:
//   * C: every load instruction of a wave covers two whole 512-byte column
//     runs (coalesced), the values are split and stored as four float16
//     planes (re hi, re lo, im hi, im lo);
//   * V': 8-wide k groups of every row, both planes.
// Slab s + 2 is loaded into registers while slab s is multiplied, and stored
// to the free buffer after slab s + 1 has been multiplied; one barrier per
// slab.
#pragma once
#include <hip/hip_runtime.h>

#include "gemm.hpp"

namespace sb2 {

struct R4Args {
  int M, ncol;               // rows i, columns c
  int kc;                    // chunk length N^2
  const _Float16* V;         // V' hi plane (row pitch ldv); lo plane at +vplane
  i64 ldv, vplane, vchunk;   // vchunk: chunk pitch within a row (multiple of 8, >= kc)
  const float* X;            // C complex float32: chunk n, column c at X + 2 (n xchunk + c kc)
  i64 xchunk;
  double* part;              // [n][i][c] complex float64
  const unsigned* vmax;      // recorded max |V'| and |C| (float bits)
  const unsigned* xmax;
};

// column tiles of 64 columns
__host__ __device__ inline int r4_tiles(const R4Args& a) { return (a.ncol + 63) / 64; }

// Workgroup (bx, by): columns 64 bx .., chunk by.  EVEN: the chunk length
// kc is even (complex pairs of C are 16-byte aligned).
template <int FS, bool EVEN>
__device__ __forceinline__ void r4_body(const R4Args& a, int bx, int by) {
  constexpr int NTH = 512, NCOL = 64, KS = 64, NKG = KS / 32;
  constexpr int FSP = (FS + 1) / 2 * 2, FH = FSP / 2;   // padded row fragments, per row half
  constexpr int LP = KS + 16;                           // 160-byte rows: 16 u bytes, u = 2 mod 4 (conflict-free fragment reads)
  static_assert((2 * 16 * FSP * (KS / 8)) % NTH == 0, "whole V' items per thread");
  constexpr int PV = 2 * 16 * FSP * (KS / 8) / NTH;     // V' items (hx8) per thread
  constexpr int PC = NCOL * KS / 2 / NTH;                // C loads (2 complex each) per thread
  __shared__ __attribute__((aligned(16))) _Float16 sV[2][2][16 * FSP][LP];
  __shared__ __attribute__((aligned(16))) _Float16 sC[2][4][NCOL][LP];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int grp = lane >> 4, lr = lane & 15;
  const int rh = w >> 2, cg = w & 3;
  const int col0 = bx * NCOL;
  // k: index within the chunk, 0 .. kc - 1
  const int k0 = 0, k1 = a.kc, K = a.kc;
  const int nslab = (k1 + KS - 1) / KS;
  const _Float16* Vz = a.V + (i64)by * a.vchunk;
  const float* Xz = a.X + 2 * ((i64)by * a.xchunk);
  const float sv = split_scale(a.vmax), sx = split_scale(a.xmax);
  const double unscale = 1.0 / ((double)sv * (double)sx);

  // ---- V' items: item u = 8-wide k group vh of combined (plane, row) R ----
  const int vh = 8 * (tid & 7), R0 = tid >> 3;
  auto vrow = [&](int u, int& pl, int& r) {
    const int R = R0 + (NTH / 8) * u;                    // < 32 FSP
    pl = R >= 16 * FSP ? 1 : 0;
    r = R - pl * 16 * FSP;
  };
  // Loads only clamp their addresses (the loaded registers are not touched
  // until they are stored, so the loads stay in flight): rows past M read row
  // M - 1 (their products land in output rows that are never written) and k
  // past the chunk reads its last 8-group; the chunk padding of V' is zero and
  // C past the chunk is zeroed when stored, so those products vanish.
  auto load_v = [&](int s, hx8 (&dst)[PV]) {
    const int ks = k0 + s * KS;
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      int pl, r;
      vrow(u, pl, r);
      const int rr = min(r, a.M - 1);
      const int kk = min(ks + vh, (int)a.vchunk - 8);
      dst[u] = *reinterpret_cast<const hx8*>(Vz + pl * a.vplane + (i64)rr * a.ldv + kk);
    }
  };
  auto store_v = [&](int buf, const hx8 (&src)[PV]) {
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      int pl, r;
      vrow(u, pl, r);
      *reinterpret_cast<hx8*>(&sV[buf][pl][r][vh]) = src[u];
    }
  };

  // ---- C items: load e of lane l covers column 8 w + 2 e + l/32, complex
  // k = 2 (l%32), 2 (l%32) + 1 of the slab ----
  const int ck = 2 * (lane & 31), chalf = lane >> 5;
  // columns past ncol read column ncol - 1 (discarded output columns)
  auto load_c = [&](int s, float4 (&dst)[PC]) {
    const int k = k0 + s * KS + ck;
#pragma unroll
    for (int e = 0; e < PC; ++e) {
      const int c = min(col0 + 8 * w + 2 * e + chalf, a.ncol - 1);
      const float* p = Xz + 2 * ((i64)c * K);
      if constexpr (EVEN) {
        dst[e] = *reinterpret_cast<const float4*>(p + 2 * min(k, K - 2));
      } else {
        const float2 x0 = *reinterpret_cast<const float2*>(p + 2 * min(k, K - 1));
        const float2 x1 = *reinterpret_cast<const float2*>(p + 2 * min(k + 1, K - 1));
        dst[e] = make_float4(x0.x, x0.y, x1.x, x1.y);
      }
    }
  };
  auto store_c = [&](int buf, int s, const float4 (&src)[PC]) {
    const int k = k0 + s * KS + ck;
    const float m0 = k < k1 ? sx : 0.f, m1 = k + 1 < k1 ? sx : 0.f;   // zero past the chunk
#pragma unroll
    for (int e = 0; e < PC; ++e) {
      const int cl = 8 * w + 2 * e + chalf;
      // packed pairs (k, k + 1) of the real and imaginary hi and lo parts
      unsigned rh, rl, ih, il;
      split_pair(src[e].x, m0, src[e].z, m1, rh, rl);
      split_pair(src[e].y, m0, src[e].w, m1, ih, il);
      *reinterpret_cast<unsigned*>(&sC[buf][0][cl][ck]) = rh;
      *reinterpret_cast<unsigned*>(&sC[buf][1][cl][ck]) = rl;
      *reinterpret_cast<unsigned*>(&sC[buf][2][cl][ck]) = ih;
      *reinterpret_cast<unsigned*>(&sC[buf][3][cl][ck]) = il;
    }
  };

  fx4 cr[FH], ci[FH];
  dx4 dr[FH], di[FH];
#pragma unroll
  for (int f = 0; f < FH; ++f) {
    cr[f] = vzero<fx4>();
    ci[f] = vzero<fx4>();
    dr[f] = vzero<dx4>();
    di[f] = vzero<dx4>();
  }

  auto compute = [&](int buf) {
#pragma unroll
    for (int kg = 0; kg < NKG; ++kg) {
      const int col = 32 * kg + 8 * grp;
      const int cl = 16 * cg + lr;
      const hx8 xrh = *reinterpret_cast<const hx8*>(&sC[buf][0][cl][col]);
      const hx8 xrl = *reinterpret_cast<const hx8*>(&sC[buf][1][cl][col]);
      const hx8 xih = *reinterpret_cast<const hx8*>(&sC[buf][2][cl][col]);
      const hx8 xil = *reinterpret_cast<const hx8*>(&sC[buf][3][cl][col]);
#pragma unroll
      for (int f = 0; f < FH; ++f) {
        if (rh * FH + f < FS) {                          // fragments past M: nothing to do
          const int row = 16 * (rh * FH + f) + lr;
          const hx8 vh8 = *reinterpret_cast<const hx8*>(&sV[buf][0][row][col]);
          const hx8 vl8 = *reinterpret_cast<const hx8*>(&sV[buf][1][row][col]);
          cr[f] = mma3(vh8, vl8, xrh, xrl, cr[f]);
          ci[f] = mma3(vh8, vl8, xih, xil, ci[f]);
        }
      }
    }
  };
  // fold the float32 sums into float64, once per two slabs (128 k: each
  // float32 partial takes 12 MFMA accumulations, against the 2^-22 relative
  // error of a split operand)
  auto fold = [&]() {
#pragma unroll
    for (int f = 0; f < FH; ++f)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        dr[f][q] += (double)cr[f][q];
        di[f][q] += (double)ci[f][q];
        cr[f][q] = 0.f;
        ci[f][q] = 0.f;
      }
  };

  // two register sets: slab s + 2 is in flight while slab s is multiplied.
  // Loads are issued unconditionally (slabs past the end read clamped,
  // in-bounds addresses and are never multiplied), so every iteration issues
  // the same memory operations and each wait covers only the set it needs.
  hx8 va[PV], vb[PV];
  float4 ca[PC], cb[PC];
  if (nslab > 0) {
    load_v(0, va);
    load_c(0, ca);
    load_v(1, vb);
    load_c(1, cb);
    store_v(0, va);
    store_c(0, 0, ca);
    __syncthreads();
  }
#pragma unroll 1
  for (int s = 0; s < nslab; s += 2) {
    // even slab s in buffer 0; set b holds slab s + 1
    load_v(s + 2, va);
    load_c(s + 2, ca);
    compute(0);
    store_v(1, vb);
    store_c(1, s + 1, cb);
    __syncthreads();
    load_v(s + 3, vb);
    load_c(s + 3, cb);
    if (s + 1 < nslab) compute(1);                    // uniform
    fold();
    store_v(0, va);
    store_c(0, s + 2, ca);
    __syncthreads();
  }

  // ---- partial sums: part[n][i][c], i = 16 f + 4 g + q ----
  const int c = col0 + 16 * cg + lr;
  if (c < a.ncol) {
    double2* out = reinterpret_cast<double2*>(a.part) + (i64)by * a.M * a.ncol + c;
#pragma unroll
    for (int f = 0; f < FH; ++f) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * (rh * FH + f) + 4 * grp + q;
        if (i < a.M) out[(i64)i * a.ncol] = make_double2(dr[f][q] * unscale, di[f][q] * unscale);
      }
    }
  }
}

template <int FS, bool EVEN>
__global__ void __launch_bounds__(512) k_r4_h16(const R4Args a) {
  r4_body<FS, EVEN>(a, blockIdx.x, blockIdx.y);
}

}  // namespace sb2
