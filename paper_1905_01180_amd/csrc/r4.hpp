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
// Workgroup: 64 columns c, 12 waves.  8 compute waves = 2 row halves x 4
// column groups (two per SIMD); wave (h, g) owns the 16 columns 16 g .. 16 g +
// 15 and the row fragments h FH .. h FH + FH - 1 of the FSP >= FS padded
// fragments.  4 producer waves (one per SIMD) stage slabs of 64 k of both
// operands in LDS, double buffered:
//   * C: every load instruction of a wave covers two whole 512-byte column
//     runs (coalesced), the values are split and stored as four float16
//     planes (re hi, re lo, im hi, im lo);
//   * V': 8-wide k groups of both planes' rows below M (rows past M only
//     reach output rows that are never written and are not loaded).
// One barrier per slab.
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

// column tiles of 64 columns; threads per workgroup
__host__ __device__ inline int r4_tiles(const R4Args& a) { return (a.ncol + 63) / 64; }
constexpr int R4_THREADS = 768;

// Workgroup (bx, by): columns 64 bx .., chunk by.  EVEN: the chunk length
// kc is even (complex pairs of C are 16-byte aligned).  The compute waves only
// read LDS and multiply; while they multiply slab s the producers split and
// store slab s + 1 (loaded two slabs earlier) into the free buffer and load
// slab s + 3, so the loads and the split of C run beside the matrix products
// instead of taking turns with them on the same waves.  Both roles run their
// own loop with the same barrier sequence (the loop unrolled twice so that
// buffers and register sets are static).
template <int FS, bool EVEN>
__device__ __forceinline__ void r4_body(const R4Args& a, int bx, int by) {
  constexpr int NCW = 8, NPW = 4, NPT = 64 * NPW;       // compute waves, producer waves / threads
  constexpr int NCOL = 64, KS = 64, NKG = KS / 32;
  constexpr int FSP = (FS + 1) / 2 * 2, FH = FSP / 2;
  constexpr int LP = KS + 16;                           // 160-byte rows: 16 u bytes, u = 2 mod 4 (conflict-free fragment reads)
  static_assert((2 * 16 * FS * (KS / 8)) % NPT == 0, "whole V' items per producer thread");
  constexpr int PV = 2 * 16 * FS * (KS / 8) / NPT;      // V' items (hx8) per producer thread (= FS)
  constexpr int PC = NCOL * KS / 2 / NPT;                // C loads (2 complex each) per producer thread
  __shared__ __attribute__((aligned(16))) _Float16 sV[2][2][16 * FSP][LP];
  __shared__ __attribute__((aligned(16))) _Float16 sC[2][4][NCOL][LP];

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col0 = bx * NCOL;
  const int K = a.kc;
  const int nslab = (K + KS - 1) / KS;
  static_assert(64 * (NCW + NPW) == R4_THREADS, "workgroup size");

  if (w >= NCW) {
    // ---- producers ----
    const int pt = tid - 64 * NCW, pw = w - NCW;
    const _Float16* Vz = a.V + (i64)by * a.vchunk;
    const float* Xz = a.X + 2 * ((i64)by * a.xchunk);
    const float sx = split_scale(a.xmax);
    // V' items: the M rows of each plane whose products are written, as
    // combined rows R = (plane) M + (row) < 2 M.  Item u of a lane is the
    // 8-wide k group vh of combined row R0 + 32 u (R0 = 8 pw + lane / 8); a
    // wave takes the NI items whose 32-row groups start below 2 M (FS - 1 or
    // FS of them, a compile-time count: no load instruction is issued for
    // rows that are never used).  Lanes past 2 M inside the last group read
    // plane 1's row M - 1 and write rows past M of plane 1; the LDS rows past
    // M of either plane are multiplied only into output rows that are never
    // written.
    const int vh = 8 * (pt & 7), R0 = pt >> 3;
    const int M = a.M;
    auto vrow = [&](int u, int& pl, int& r) {
      const int R = R0 + (NPT / 8) * u;
      pl = R >= M ? 1 : 0;
      r = min(R - pl * M, 16 * FSP - 1);
    };
    // Loads only clamp their addresses: k past the chunk reads its last
    // 8-group (the chunk padding is zero), slabs past the end are never
    // multiplied.  Each load is the chunk's base plus a 32-bit byte offset
    // (both planes of V' span under 1.1e9 bytes for N <= 128).
    unsigned vro[PV];
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      int pl, r;
      vrow(u, pl, r);
      vro[u] = 2u * (unsigned)(pl * a.vplane + (i64)min(r, M - 1) * a.ldv);
    }
    auto load_v = [&](auto NIc, int s, hx8 (&dst)[PV]) {
      const unsigned ko = 2u * (unsigned)min(s * KS + vh, (int)a.vchunk - 8);
      const char* base = reinterpret_cast<const char*>(Vz);
#pragma unroll
      for (int u = 0; u < decltype(NIc)::value; ++u) dst[u] = *reinterpret_cast<const hx8*>(base + (vro[u] + ko));
    };
    auto store_v = [&](auto NIc, int buf, const hx8 (&src)[PV]) {
#pragma unroll
      for (int u = 0; u < decltype(NIc)::value; ++u) {
        int pl, r;
        vrow(u, pl, r);
        *reinterpret_cast<hx8*>(&sV[buf][pl][r][vh]) = src[u];
      }
    };
    // C load e of a producer lane: column 16 pw + 2 e + lane / 32, complex
    // k = 2 (lane % 32), + 1 of the slab; uniform column base per load
    // (columns past ncol read column ncol - 1)
    const int ck = 2 * (lane & 31), chalf = lane >> 5;
    auto load_c = [&](int s, float4 (&dst)[PC]) {
      const int k = s * KS + ck;
#pragma unroll
      for (int e = 0; e < PC; ++e) {
        const int ce = col0 + 16 * pw + 2 * e;
        const char* base = reinterpret_cast<const char*>(Xz + 2 * ((i64)min(ce, a.ncol - 1) * K));
        const unsigned co = ce + 1 < a.ncol ? (unsigned)chalf * 8u * (unsigned)K : 0u;
        if constexpr (EVEN) {
          dst[e] = *reinterpret_cast<const float4*>(base + (co + 8u * (unsigned)min(k, K - 2)));
        } else {
          const float2 x0 = *reinterpret_cast<const float2*>(base + (co + 8u * (unsigned)min(k, K - 1)));
          const float2 x1 = *reinterpret_cast<const float2*>(base + (co + 8u * (unsigned)min(k + 1, K - 1)));
          dst[e] = make_float4(x0.x, x0.y, x1.x, x1.y);
        }
      }
    };
    auto store_c = [&](int buf, int s, const float4 (&src)[PC]) {
      const int k = s * KS + ck;
      const float m0 = k < K ? sx : 0.f, m1 = k + 1 < K ? sx : 0.f;   // zero past the chunk
#pragma unroll
      for (int e = 0; e < PC; ++e) {
        const int cl = 16 * pw + 2 * e + chalf;
        unsigned rhi, rlo, ihi, ilo;
        split_pair(src[e].x, m0, src[e].z, m1, rhi, rlo);
        split_pair(src[e].y, m0, src[e].w, m1, ihi, ilo);
        *reinterpret_cast<unsigned*>(&sC[buf][0][cl][ck]) = rhi;
        *reinterpret_cast<unsigned*>(&sC[buf][1][cl][ck]) = rlo;
        *reinterpret_cast<unsigned*>(&sC[buf][2][cl][ck]) = ihi;
        *reinterpret_cast<unsigned*>(&sC[buf][3][cl][ck]) = ilo;
      }
    };
    // set a holds even slabs, set b odd ones, each loaded three slabs ahead
    // of its use; every step issues the same loads, so each wait covers only
    // the set being stored.  (Scheduling fences: the compiler would otherwise
    // hoist the register-only split of the next set above the barrier and wait
    // for its loads a slab early.)
    auto produce = [&](auto NIc) {
      hx8 va[PV], vb[PV];
      float4 ca[PC], cb[PC];
      if (nslab > 0) {
        load_v(NIc, 0, va);
        load_c(0, ca);
        load_v(NIc, 1, vb);
        load_c(1, cb);
        store_v(NIc, 0, va);
        store_c(0, 0, ca);
        load_v(NIc, 2, va);
        load_c(2, ca);
      }
#pragma unroll 1
      for (int s = 0; s < nslab; s += 2) {
        __syncthreads();                                // slab s in buffer 0; buffer 1 free
        __builtin_amdgcn_sched_barrier(0);
        store_v(NIc, 1, vb);
        store_c(1, s + 1, cb);
        load_v(NIc, s + 3, vb);
        load_c(s + 3, cb);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();                                // slab s + 1 in buffer 1; buffer 0 free
        __builtin_amdgcn_sched_barrier(0);
        store_v(NIc, 0, va);
        store_c(0, s + 2, ca);
        load_v(NIc, s + 4, va);
        load_c(s + 4, ca);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    // items of this wave (wave-uniform): FS - 1 or FS, as M > 16 (FS - 1)
    const int ni = (2 * M - 8 * pw + 31) / 32;
    if (ni >= PV) produce(std::integral_constant<int, PV>{});
    else produce(std::integral_constant<int, PV - 1>{});
    return;
  }

  // ---- compute waves: row half RH (wave-uniform) as a template parameter,
  // so that the fragments past M drop out at compile time ----
  const int grp = lane >> 4, lr = lane & 15;
  const int cg = w & 3;
  const float sv = split_scale(a.vmax), sx = split_scale(a.xmax);
  const double unscale = 1.0 / ((double)sv * (double)sx);
  auto run = [&](auto rhc) {
    constexpr int RH = decltype(rhc)::value;
    constexpr int NF = FS - RH * FH <= 0 ? 0 : FS - RH * FH < FH ? FS - RH * FH : FH;   // fragments of this half
    fx4 cr[FH], ci[FH];
    dx4 dr[FH], di[FH];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
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
        for (int f = 0; f < NF; ++f) {
          const int row = 16 * (RH * FH + f) + lr;
          const hx8 vh8 = *reinterpret_cast<const hx8*>(&sV[buf][0][row][col]);
          const hx8 vl8 = *reinterpret_cast<const hx8*>(&sV[buf][1][row][col]);
          cr[f] = mma3(vh8, vl8, xrh, xrl, cr[f]);
          ci[f] = mma3(vh8, vl8, xih, xil, ci[f]);
        }
      }
    };
    // fold the float32 sums into float64 once per two slabs
    auto fold = [&]() {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          dr[f][q] += (double)cr[f][q];
          di[f][q] += (double)ci[f][q];
          cr[f][q] = 0.f;
          ci[f][q] = 0.f;
        }
    };
#pragma unroll 1
    for (int s = 0; s < nslab; s += 2) {
      __syncthreads();
      compute(0);
      __syncthreads();
      if (s + 1 < nslab) compute(1);                    // uniform
      fold();
    }
    const int c = col0 + 16 * cg + lr;
    if (c < a.ncol) {
      double2* out = reinterpret_cast<double2*>(a.part) + (i64)by * a.M * a.ncol + c;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * (RH * FH + f) + 4 * grp + q;
          if (i < a.M) out[(i64)i * a.ncol] = make_double2(dr[f][q] * unscale, di[f][q] * unscale);
        }
      }
    }
  };
  if ((w >> 2) == 0) run(std::integral_constant<int, 0>{});
  else run(std::integral_constant<int, 1>{});
}

template <int FS, bool EVEN>
__global__ void __launch_bounds__(R4_THREADS) k_r4_h16(const R4Args a) {
  r4_body<FS, EVEN>(a, blockIdx.x, blockIdx.y);
}

}  // namespace sb2
