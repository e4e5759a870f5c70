// Streaming contraction kernel for the four stages of the second-Born chain.
//
//   out(m, n) = sum_k P(m, k) Q(n, k)        (both operands K-contiguous)
//
// One operand is "shared": a tile of 16*FS of its rows is staged in LDS (in
// K slabs of KS) and used by every wave of the workgroup.  The other operand is
// "streamed": each of the NW waves owns 16*FX of its rows and loads them from
// global memory straight into MFMA fragment registers, K-vector by K-vector,
// prefetching one K-group ahead; the streamed data is never staged in LDS.
// SA = true: the shared operand supplies the output rows (P = shared, Q =
// streamed); SA = false: the streamed operand supplies the rows.
//
// K order inside one MFMA: lane group g = lane/16 holds the K-vector
// k0 + KV g .. k0 + KV g + KV - 1 of its row for BOTH operands, and the four
// (f32/f64: KV = 4, one MFMA per vector element) or one (f16: KV = 8, one
// 16x16x32 MFMA) instruction(s) per K-group consume those vectors.  The sum
// over a K-group is the same set of products in a permuted order.
//
// Precisions (PK): float64 and float32 operands are used as stored.  Split
// float16 (PK_H16): complex operands are stored as float32 and split in
// registers (streamed) or when staged into LDS (shared): x 2^e = hi + lo, with
// hi, lo float16 and 2^e a power of two from the operand's recorded max |x|
// (so |x 2^e| < 2^14); real operands (the interaction tensor) arrive pre-split
// as two float16 planes with the same rule.  Each real product is
// hi*hi + hi*lo + lo*hi on the f16 matrix cores with float32 accumulation.
#pragma once
#include <hip/hip_runtime.h>

#include "gemm.hpp"

namespace sb2 {

enum { PK_F64 = 0, PK_F32 = 1, PK_H16 = 2 };

template <int PK> struct ST;
template <> struct ST<PK_F64> { using T = double; using acc = dx4; using L = double; static constexpr int KV = 4; };
template <> struct ST<PK_F32> { using T = float; using acc = fx4; using L = float; static constexpr int KV = 4; };
template <> struct ST<PK_H16> { using T = float; using acc = fx4; using L = _Float16; static constexpr int KV = 8; };

struct StreamArgs {
  int M, N, K;
  int kchunk;              // split-K chunk; blockIdx.z picks [z kchunk, (z+1) kchunk)
  int nbl;                 // batch index z = bh nbl + bl (blockIdx.y)
  int tiles_m;             // blockIdx.x = tm + tiles_m tn
  // shared operand: element (s, k) at S + s sSs + k (k contiguous); pre-split
  // real float16 operands keep their lo plane at +sSplane elements
  const void* S; i64 sSs, sSbh, sSbl, sSplane;
  // streamed operand: element (x, k) at X + x sXx + k
  const void* X; i64 sXx, sXbh, sXbl, sXplane;
  // output element (m, n) at C + moff(m) + n sCn (complex unless out_real),
  // moff(m) = m sCm, or (m / Mlo) sCmh + (m % Mlo) sCm when Mlo > 0
  void* C; i64 sCm, sCn, sCbh, sCbl, sCz;
  int Mlo; i64 sCmh;
  int kpromote;            // ACC64: fold float32 partials into float64 every kpromote K-groups
  const unsigned* smax;    // H16: scale sources (max |x| as float bits)
  const unsigned* xmax;
  unsigned* cmax;          // H16 producers: raised to max |out|
  void* trash;             // >= 64 x 16 bytes: sink of out-of-range tile stores (stream1_body)
};

// The pointer unchanged, but opaque to the optimiser (an empty asm statement
// on its value): a store through a selected address stays one unconditional
// store instead of being split into branches.
template <typename P>
__device__ __forceinline__ __attribute__((address_space(1))) P* opaque(P* p) {
  unsigned long long a = reinterpret_cast<unsigned long long>(p);
  asm volatile("" : "+v"(a));
  return reinterpret_cast<__attribute__((address_space(1))) P*>(a);   // global memory
}

template <typename V, int N_>
__device__ __forceinline__ void zero_arr(V (&a)[N_]) {
#pragma unroll
  for (int i = 0; i < N_; ++i) a[i] = vzero<V>();
}

// complex (or real) multiply-accumulate of one fragment pair
template <bool AC, bool BC, typename S, typename V>
__device__ __forceinline__ void cmac(V& cr, V& ci, S ar, S ai, S br, S bi) {
  cr = mma(ar, br, cr);
  if constexpr (AC && BC) {
    cr = mma(-ai, bi, cr);
    ci = mma(ar, bi, ci);
    ci = mma(ai, br, ci);
  } else if constexpr (AC) {
    ci = mma(ai, br, ci);
  } else if constexpr (BC) {
    ci = mma(ar, bi, ci);
  }
}

template <bool AC, bool BC>
__device__ __forceinline__ void cmac3(fx4& cr, fx4& ci, hx8 arh, hx8 arl, hx8 aih, hx8 ail, hx8 brh, hx8 brl,
                                      hx8 bih, hx8 bil) {
  cr = mma3(arh, arl, brh, brl, cr);
  if constexpr (AC && BC) {
    cr = mma3(-aih, -ail, bih, bil, cr);
    ci = mma3(arh, arl, bih, bil, ci);
    ci = mma3(aih, ail, brh, brl, ci);
  } else if constexpr (AC) {
    ci = mma3(aih, ail, brh, brl, ci);
  } else if constexpr (BC) {
    ci = mma3(arh, arl, bih, bil, ci);
  }
}

__device__ __forceinline__ void split16(float x, _Float16& hi, _Float16& lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (float)hi);
}

// Kernel layout of the launch grid:
//   grid.x = tiles of the shared operand (ts) x npersist workgroups per shared tile;
//   a workgroup keeps its shared tile resident and walks streamed tiles
//   tx = p, p + npersist, ... (single-slab case, K <= KS), or handles one
//   streamed tile while walking K slabs (multi-slab / split-K case);
//   grid.y = batch, grid.z = split-K chunk.
template <int PK, bool SA, bool SC, bool XC, int FS, int FX, int NW, int KS, bool ACC64, typename OutT>
__device__ __forceinline__ void stream_body(const StreamArgs& g, int bx, int by, int bzz, int npersist_arg) {
  using Tr = ST<PK>;
  using T = typename Tr::T;
  using LT = typename Tr::L;
  using acc_t = typename Tr::acc;
  constexpr bool H = PK == PK_H16;
  constexpr int KV = Tr::KV, KG = 4 * KV;
  constexpr int NT = 64 * NW;
  constexpr int SR = 16 * FS;
  constexpr int XW = 16 * FX, XT = XW * NW;
  constexpr int NPL = (H ? 2 : 1) * (SC ? 2 : 1);
  constexpr int LPB0 = KS * (int)sizeof(LT);
  // 16-byte fragment reads (split float16): pitch 16 u bytes with u = 2 mod 4;
  // element reads (float32, float64): pitch 16 mod 128 bytes
  constexpr int PADB = H ? ((32 - LPB0 % 64) + 64) % 64 : ((16 - LPB0 % 128) + 128) % 128;
  constexpr int LP = KS + PADB / (int)sizeof(LT);
  constexpr int SE = SC ? 2 : 1, XE = XC ? 2 : 1;     // scalars per element
  static_assert(KS % KG == 0, "slab must hold whole K-groups");

  __shared__ __attribute__((aligned(16))) LT sS[NPL][SR][LP];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int grp = lane >> 4, lr = lane & 15;
  const int ts = bx % g.tiles_m, pp = bx / g.tiles_m;   // tiles_m = shared tiles
  const int s0 = ts * SR;
  const int slim = SA ? g.M : g.N;
  const int xlim = SA ? g.N : g.M;
  const int tiles_x = (xlim + XT - 1) / XT;
  const int bz = by, bh = bz / g.nbl, bl = bz - bh * g.nbl;
  const int kbeg = bzz * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const bool single = kend - kbeg <= KS;
  const int npersist = npersist_arg;

  const i64 sbatch = (i64)bh * g.sSbh + (i64)bl * g.sSbl;
  const i64 xbatch = (i64)bh * g.sXbh + (i64)bl * g.sXbl;
  float ss = 1.f, sx = 1.f;
  if constexpr (H) {
    ss = split_scale(g.smax);
    sx = split_scale(g.xmax);
  }
  OutT* Cb = reinterpret_cast<OutT*>(g.C) + 2 * ((i64)bh * g.sCbh + (i64)bl * g.sCbl + (i64)bzz * g.sCz);
  const double unscale = H ? 1.0 / ((double)ss * (double)sx) : 1.0;

  acc_t cr[FS][FX], ci[FS][FX];
  dx4 dr[ACC64 ? FS : 1][ACC64 ? FX : 1], di[ACC64 ? FS : 1][ACC64 ? FX : 1];
  T xr[FX][KV], xi[FX][KV], nxr[FX][KV], nxi[FX][KV];
  hx8 xph[FX], xpl[FX], nxph[FX], nxpl[FX];
  float mx = 0.f;

  // ---- streamed operand: one K-group (KG) of this wave's 16 FX rows ----
  auto load_x = [&](int x0, int kg0, T (&xr)[FX][KV], T (&xi)[FX][KV], hx8 (&xph)[FX], hx8 (&xpl)[FX]) {
    const int k = kg0 + KV * grp;
    const bool full = kg0 + KG <= kend;
#pragma unroll
    for (int f = 0; f < FX; ++f) {
      const int x = x0 + f * 16 + lr;
      const bool xv = x < xlim;
      if constexpr (H && !XC) {
        const _Float16* p = reinterpret_cast<const _Float16*>(g.X) + xbatch + (i64)x * g.sXx + k;
        hx8 vh, vl;
#pragma unroll
        for (int e = 0; e < 8; ++e) { vh[e] = (_Float16)0.f; vl[e] = (_Float16)0.f; }
        if (xv) {
          if (full) {
            vh = *reinterpret_cast<const hx8*>(p);
            vl = *reinterpret_cast<const hx8*>(p + g.sXplane);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (k + e < kend) { vh[e] = p[e]; vl[e] = p[g.sXplane + e]; }
          }
        }
        xph[f] = vh;
        xpl[f] = vl;
      } else {
        const T* p = reinterpret_cast<const T*>(g.X) + XE * (xbatch + (i64)x * g.sXx + k);
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          T re = T(0), im = T(0);
          if (xv && (full || k + e < kend)) {
            if constexpr (XC) {
              typedef T t2 __attribute__((ext_vector_type(2)));
              const t2 v = *reinterpret_cast<const t2*>(p + 2 * e);
              re = v[0];
              im = v[1];
            } else {
              re = p[e];
            }
          }
          xr[f][e] = re;
          if constexpr (XC) xi[f][e] = im;
        }
      }
    }
  };

  // ---- shared slab staging: all loads of a batch issued before any use ----
  auto load_slab = [&](int ks0) {
    if constexpr (H && !SC) {
      const _Float16* Sb = reinterpret_cast<const _Float16*>(g.S) + sbatch;
      constexpr int C8 = KS / 8;
      constexpr int ITEMS = SR * C8, PER = (ITEMS + NT - 1) / NT;
      hx8 vh[PER], vl[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int L = tid + u * NT;
        const int r = L / C8, c = (L - (L / C8) * C8) * 8;
        const int srow = s0 + r, k = ks0 + c;
#pragma unroll
        for (int e = 0; e < 8; ++e) { vh[u][e] = (_Float16)0.f; vl[u][e] = (_Float16)0.f; }
        if (L < ITEMS && srow < slim) {
          const _Float16* p = Sb + (i64)srow * g.sSs + k;
          if (k + 8 <= kend) {
            vh[u] = *reinterpret_cast<const hx8*>(p);
            vl[u] = *reinterpret_cast<const hx8*>(p + g.sSplane);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (k + e < kend) { vh[u][e] = p[e]; vl[u][e] = p[g.sSplane + e]; }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int L = tid + u * NT;
        if (L < ITEMS) {
          const int r = L / C8, c = (L - (L / C8) * C8) * 8;
          *reinterpret_cast<hx8*>(&sS[0][r][c]) = vh[u];
          *reinterpret_cast<hx8*>(&sS[1][r][c]) = vl[u];
        }
      }
    } else {
      const T* Sb = reinterpret_cast<const T*>(g.S) + SE * sbatch;
      constexpr int ITEMS = SR * KS, PER = (ITEMS + NT - 1) / NT;
      constexpr int BATCH = 8, NB = (PER + BATCH - 1) / BATCH;
#pragma unroll 1
      for (int bt = 0; bt < NB; ++bt) {
        T re[BATCH], im[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          const int L = tid + (bt * BATCH + u) * NT;
          const int r = L / KS, c = L - (L / KS) * KS;
          const int srow = s0 + r, k = ks0 + c;
          re[u] = T(0);
          im[u] = T(0);
          if (L < ITEMS && srow < slim && k < kend) {
            const T* p = Sb + SE * ((i64)srow * g.sSs + k);
            if constexpr (SC) {
              typedef T t2 __attribute__((ext_vector_type(2)));
              const t2 v = *reinterpret_cast<const t2*>(p);
              re[u] = v[0];
              im[u] = v[1];
            } else {
              re[u] = p[0];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          const int L = tid + (bt * BATCH + u) * NT;
          if (L < ITEMS) {
            const int r = L / KS, c = L - (L / KS) * KS;
            if constexpr (H) {
              split16(re[u] * ss, sS[0][r][c], sS[1][r][c]);
              if constexpr (SC) split16(im[u] * ss, sS[2][r][c], sS[3][r][c]);
            } else {
              sS[0][r][c] = re[u];
              if constexpr (SC) sS[1][r][c] = im[u];
            }
          }
        }
      }
    }
  };

  // ---- one K-group of MFMAs on the current streamed registers ----
  auto compute = [&](int kl) {
    if constexpr (H) {
      hx8 xrh[FX], xrl[FX], xih[FX], xil[FX];
#pragma unroll
      for (int f = 0; f < FX; ++f) {
        if constexpr (XC) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float a = xr[f][e] * sx, b = xi[f][e] * sx;
            const _Float16 ah = (_Float16)a, bh = (_Float16)b;
            xrh[f][e] = ah;
            xrl[f][e] = (_Float16)(a - (float)ah);
            xih[f][e] = bh;
            xil[f][e] = (_Float16)(b - (float)bh);
          }
        } else {
          xrh[f] = xph[f];
          xrl[f] = xpl[f];
          xih[f] = xph[f];
          xil[f] = xpl[f];
        }
      }
#pragma unroll
      for (int i = 0; i < FS; ++i) {
        const int row = i * 16 + lr;
        const hx8 srh = *reinterpret_cast<const hx8*>(&sS[0][row][kl + 8 * grp]);
        const hx8 srl = *reinterpret_cast<const hx8*>(&sS[1][row][kl + 8 * grp]);
        hx8 sih = srh, sil = srl;
        if constexpr (SC) {
          sih = *reinterpret_cast<const hx8*>(&sS[NPL - 2][row][kl + 8 * grp]);
          sil = *reinterpret_cast<const hx8*>(&sS[NPL - 1][row][kl + 8 * grp]);
        }
#pragma unroll
        for (int f = 0; f < FX; ++f) {
          if constexpr (SA)
            cmac3<SC, XC>(cr[i][f], ci[i][f], srh, srl, sih, sil, xrh[f], xrl[f], xih[f], xil[f]);
          else
            cmac3<XC, SC>(cr[i][f], ci[i][f], xrh[f], xrl[f], xih[f], xil[f], srh, srl, sih, sil);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < FS; ++i) {
        const int row = i * 16 + lr;
        T sr[4], si[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          sr[e] = sS[0][row][kl + 4 * grp + e];
          si[e] = SC ? sS[NPL - 1][row][kl + 4 * grp + e] : T(0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
          for (int f = 0; f < FX; ++f) {
            const T xre = xr[f][e];
            const T xim = XC ? xi[f][e] : T(0);
            if constexpr (SA) cmac<SC, XC>(cr[i][f], ci[i][f], sr[e], si[e], xre, xim);
            else cmac<XC, SC>(cr[i][f], ci[i][f], xre, xim, sr[e], si[e]);
          }
        }
      }
    }
  };

  auto shift_regs = [&]() {
#pragma unroll
    for (int f = 0; f < FX; ++f) {
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        xr[f][e] = nxr[f][e];
        if constexpr (XC) xi[f][e] = nxi[f][e];
      }
      if constexpr (H && !XC) {
        xph[f] = nxph[f];
        xpl[f] = nxpl[f];
      }
    }
  };

  auto fold = [&](bool final_) {
    if constexpr (ACC64) {
#pragma unroll
      for (int i = 0; i < FS; ++i)
#pragma unroll
        for (int f = 0; f < FX; ++f)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            dr[i][f][q] += (double)cr[i][f][q];
            di[i][f][q] += (double)ci[i][f][q];
            cr[i][f][q] = 0;
            ci[i][f][q] = 0;
          }
    }
    (void)final_;
  };

  auto reset = [&]() {
#pragma unroll
    for (int i = 0; i < FS; ++i) {
      zero_arr(cr[i]);
      zero_arr(ci[i]);
      if constexpr (ACC64) {
        zero_arr(dr[i]);
        zero_arr(di[i]);
      }
    }
  };

  auto epilogue = [&](int x0) {
#pragma unroll
    for (int i = 0; i < FS; ++i) {
#pragma unroll
      for (int f = 0; f < FX; ++f) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int fr = frag_row<T>(grp, q);
          const int m = SA ? s0 + i * 16 + fr : x0 + f * 16 + fr;
          const int n = SA ? x0 + f * 16 + lr : s0 + i * 16 + lr;
          if (m < g.M && n < g.N) {
            double re, im;
            if constexpr (ACC64) { re = dr[i][f][q]; im = di[i][f][q]; }
            else { re = (double)cr[i][f][q]; im = (double)ci[i][f][q]; }
            re *= unscale;
            im *= unscale;
            i64 om;
            if (g.Mlo > 0) {
              const int mh = m / g.Mlo;
              om = (i64)mh * g.sCmh + (i64)(m - mh * g.Mlo) * g.sCm;
            } else {
              om = (i64)m * g.sCm;
            }
            typedef OutT o2 __attribute__((ext_vector_type(2)));
            o2 v;
            v[0] = (OutT)re;
            v[1] = (OutT)im;
            *reinterpret_cast<o2*>(Cb + 2 * (om + (i64)n * g.sCn)) = v;
            if constexpr (H) mx = fmaxf(mx, fmaxf(fabsf((float)re), fabsf((float)im)));
          }
        }
      }
    }
  };

  if (kend > kbeg) {
    if (single) {
      // shared tile resident; walk the streamed tiles of this workgroup
      load_slab(kbeg);
      __syncthreads();
      int tx = pp;
      if (tx < tiles_x) load_x(tx * XT + w * XW, kbeg, xr, xi, xph, xpl);
      for (; tx < tiles_x; tx += npersist) {
        const int x0 = tx * XT + w * XW;
        const int txn = tx + npersist;
        reset();
        int gcount = 0;
        for (int kg0 = kbeg; kg0 < kend; kg0 += KG) {
          const bool more = kg0 + KG < kend;
          if (more) load_x(x0, kg0 + KG, nxr, nxi, nxph, nxpl);
          else if (txn < tiles_x) load_x(txn * XT + w * XW, kbeg, nxr, nxi, nxph, nxpl);
          compute(kg0 - kbeg);
          if (more || txn < tiles_x) shift_regs();
          ++gcount;
          if constexpr (ACC64) {
            if (gcount % g.kpromote == 0) fold(false);
          }
        }
        fold(true);
        epilogue(x0);
      }
    } else {
      // one streamed tile, K walked in slabs of the shared operand
      const int tx = pp;
      if (tx < tiles_x) {
        const int x0 = tx * XT + w * XW;
        reset();
        load_x(x0, kbeg, xr, xi, xph, xpl);
        int gcount = 0;
        for (int ks0 = kbeg; ks0 < kend; ks0 += KS) {
          __syncthreads();
          load_slab(ks0);
          __syncthreads();
          const int kse = min(kend, ks0 + KS);
          for (int kg0 = ks0; kg0 < kse; kg0 += KG) {
            const bool more = kg0 + KG < kend;
            if (more) load_x(x0, kg0 + KG, nxr, nxi, nxph, nxpl);
            compute(kg0 - ks0);
            if (more) shift_regs();
            ++gcount;
            if constexpr (ACC64) {
              if (gcount % g.kpromote == 0) fold(false);
            }
          }
        }
        fold(true);
        epilogue(x0);
      }
    }
  }
  if constexpr (H) {
    if (g.cmax) {
      mx = wave_max(mx);
      if (lane == 0 && mx > 0.f) atomicMax(g.cmax, __float_as_uint(mx));
    }
  }
}

template <int PK, bool SA, bool SC, bool XC, int FS, int FX, int NW, int KS, bool ACC64, typename OutT>
__global__ void __launch_bounds__(64 * NW) k_stream(const StreamArgs g) {
  stream_body<PK, SA, SC, XC, FS, FX, NW, KS, ACC64, OutT>(g, blockIdx.x, blockIdx.y, blockIdx.z,
                                                            (int)(gridDim.x / g.tiles_m));
}


}  // namespace sb2

namespace sb2 {

// ---------------------------------------------------------------------------
// Single-slab variant (K <= KS) with whole-tile register double buffering.
// Each wave streams one 16-row fragment (FX = 1); all K-groups of its next
// tile are loaded into a second register set while the current tile is
// multiplied, so a wave keeps a full tile of loads in flight.  The shared
// operand stays resident in LDS for the workgroup's whole walk over tiles.
// ---------------------------------------------------------------------------
template <int PK, bool XC, int NKG>
struct XTile {
  using T = typename ST<PK>::T;
  static constexpr int KV = ST<PK>::KV;
  T re[NKG][KV];
  T im[XC ? NKG : 1][KV];
  hx8 ph[(PK == PK_H16 && !XC) ? NKG : 1], pl[(PK == PK_H16 && !XC) ? NKG : 1];
};

template <int PK, bool SA, bool SC, bool XC, int FS, int NW, int KS, typename OutT>
__device__ __forceinline__ void stream1_body(const StreamArgs& g, int bx, int by, int npersist) {
  using Tr = ST<PK>;
  using T = typename Tr::T;
  using LT = typename Tr::L;
  using acc_t = typename Tr::acc;
  constexpr bool H = PK == PK_H16;
  constexpr int KV = Tr::KV, KG = 4 * KV, NKG = KS / KG;
  // the streamed rows are buffered in two super-groups of SGQ K-groups each
  constexpr int SGQ = NKG / 2;
  static_assert(NKG % 2 == 0, "two super-groups per tile");
  using XT_ = XTile<PK, XC, SGQ>;
  constexpr int NT = 64 * NW;
  constexpr int SR = 16 * FS;
  constexpr int XT = 16 * NW;
  constexpr int NPL = (H ? 2 : 1) * (SC ? 2 : 1);
  constexpr int LPB0 = KS * (int)sizeof(LT);
  // 16-byte fragment reads (split float16): pitch 16 u bytes with u = 2 mod 4;
  // element reads (float32, float64): pitch 16 mod 128 bytes
  constexpr int PADB = H ? ((32 - LPB0 % 64) + 64) % 64 : ((16 - LPB0 % 128) + 128) % 128;
  constexpr int LP = KS + PADB / (int)sizeof(LT);
  constexpr int SE = SC ? 2 : 1, XE = XC ? 2 : 1;
  static_assert(KS % KG == 0, "slab must hold whole K-groups");

  __shared__ __attribute__((aligned(16))) LT sS[NPL][SR][LP];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int grp = lane >> 4, lr = lane & 15;
  // workgroup bx -> (shared-operand tile ts, first streamed tile pp).  Launch
  // order deals workgroups to the 8 XCDs round-robin (bx % 8); when npersist
  // is a multiple of 8, all tiles_m workgroups of one pp (which stream the
  // same X tiles) are placed on one XCD, whose L2 then serves the X re-reads
  int ts, pp;
  if (npersist % 8 == 0) {
    const int slot = bx >> 3;
    ts = slot % g.tiles_m;
    pp = 8 * (slot / g.tiles_m) + (bx & 7);
  } else {
    ts = bx % g.tiles_m;
    pp = bx / g.tiles_m;
  }
  const int s0 = ts * SR;
  const int slim = SA ? g.M : g.N;
  const int xlim = SA ? g.N : g.M;
  const int tiles_x = (xlim + XT - 1) / XT;
  const int bz = by, bh = bz / g.nbl, bl = bz - bh * g.nbl;
  const int kbeg = 0, kend = g.K;
  const i64 sbatch = (i64)bh * g.sSbh + (i64)bl * g.sSbl;
  const i64 xbatch = (i64)bh * g.sXbh + (i64)bl * g.sXbl;
  float ss = 1.f, sx = 1.f;
  if constexpr (H) {
    ss = split_scale(g.smax);
    sx = split_scale(g.xmax);
  }
  OutT* Cb = reinterpret_cast<OutT*>(g.C) + 2 * ((i64)bh * g.sCbh + (i64)bl * g.sCbl);
  const double unscale = H ? 1.0 / ((double)ss * (double)sx) : 1.0;
  float mx = 0.f;

  // ---- shared operand: staged once ----
  {
    const T* Sb = reinterpret_cast<const T*>(g.S) + SE * sbatch;
    constexpr int ITEMS = SR * KS, PER = (ITEMS + NT - 1) / NT;
    constexpr int BATCH = 8, NB = (PER + BATCH - 1) / BATCH;
#pragma unroll 1
    for (int bt = 0; bt < NB; ++bt) {
      T re[BATCH], im[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int L = tid + (bt * BATCH + u) * NT;
        const int r = L / KS, c = L - (L / KS) * KS;
        const int srow = s0 + r, k = kbeg + c;
        re[u] = T(0);
        im[u] = T(0);
        if (L < ITEMS && srow < slim && k < kend) {
          const T* p = Sb + SE * ((i64)srow * g.sSs + k);
          if constexpr (SC) {
            typedef T t2 __attribute__((ext_vector_type(2)));
            const t2 v = *reinterpret_cast<const t2*>(p);
            re[u] = v[0];
            im[u] = v[1];
          } else {
            re[u] = p[0];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int L = tid + (bt * BATCH + u) * NT;
        if (L < ITEMS) {
          const int r = L / KS, c = L - (L / KS) * KS;
          if constexpr (H) {
            split16(re[u] * ss, sS[0][r][c], sS[1][r][c]);
            if constexpr (SC) split16(im[u] * ss, sS[2][r][c], sS[3][r][c]);
          } else {
            sS[0][r][c] = re[u];
            if constexpr (SC) sS[1][r][c] = im[u];
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- streamed tile loads (all K-groups) ----
  // Rows past the end are clamped to the last row (a valid address) and their
  // values zeroed; K-groups are either complete (no per-element test) or the
  // single tail group, whose columns are clamped to K-1 and zeroed.
  const char* Xb = reinterpret_cast<const char*>(g.X);
  auto load_sg = [&](int tx, int half, XT_& t) {
    const int x = tx * XT + w * 16 + lr;
    const bool xv = x < xlim;
    const bool edge = tx * XT + XT > xlim;                  // uniform per workgroup
    const int xc = xv ? x : xlim - 1;
#pragma unroll
    for (int q = 0; q < SGQ; ++q) {
      const int kg0 = kbeg + (half * SGQ + q) * KG;
      if (kg0 >= kend) continue;                            // uniform: whole group past K
      const int k = kg0 + KV * grp;
      if constexpr (H && !XC) {
        // Whole 8-element groups at clamped addresses, never masked, so the
        // loads stay in flight until the products use them: the row pitch
        // sXx is a multiple of 8 with zero padding past K, the shared operand
        // is zero for k >= K (so any finite value there contributes nothing),
        // and rows past the end read the last row (their outputs are not stored).
        const _Float16* p = reinterpret_cast<const _Float16*>(Xb) + xbatch + (i64)xc * g.sXx;
        const int kc = min(k, (int)g.sXx - 8);
        t.ph[q] = *reinterpret_cast<const hx8*>(p + kc);
        t.pl[q] = *reinterpret_cast<const hx8*>(p + g.sXplane + kc);
      } else {
        const T* p = reinterpret_cast<const T*>(Xb) + XE * (xbatch + (i64)xc * g.sXx);
        if (kg0 + KG <= kend) {
#pragma unroll
          for (int e = 0; e < KV; ++e) {
            if constexpr (XC) {
              typedef T t2 __attribute__((ext_vector_type(2)));
              const t2 v = *reinterpret_cast<const t2*>(p + 2 * (k + e));
              t.re[q][e] = v[0];
              t.im[q][e] = v[1];
            } else {
              t.re[q][e] = p[k + e];
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < KV; ++e) {
            const int kk = min(k + e, kend - 1);
            const bool ok = k + e < kend;
            if constexpr (XC) {
              typedef T t2 __attribute__((ext_vector_type(2)));
              const t2 v = *reinterpret_cast<const t2*>(p + 2 * kk);
              t.re[q][e] = ok ? v[0] : T(0);
              t.im[q][e] = ok ? v[1] : T(0);
            } else {
              const T v = p[kk];
              t.re[q][e] = ok ? v : T(0);
            }
          }
        }
        if (edge && !xv) {
#pragma unroll
          for (int e = 0; e < KV; ++e) {
            t.re[q][e] = T(0);
            if constexpr (XC) t.im[q][e] = T(0);
          }
        }
      }
    }
  };

  // output offsets: the part that does not change from tile to tile
  // SA: rows m = s0 + 16 i + fr(q) are fixed, columns n = x0 + lr move with the tile
  // SB: columns n = s0 + 16 i + lr are fixed, rows m = x0 + fr(q) move with the tile
  i64 fixoff[SA ? 4 : 1];
  i64 fixstep = 0;                                          // per fragment i
  if constexpr (SA) {
#pragma unroll
    for (int q = 0; q < 4; ++q) fixoff[q] = (i64)(s0 + frag_row<T>(grp, q)) * g.sCm;
    fixstep = (i64)16 * g.sCm;
  } else {
    fixoff[0] = (i64)(s0 + lr) * g.sCn;
    fixstep = (i64)16 * g.sCn;
  }

  // ---- multiply one super-group into the accumulators ----
  acc_t cr[FS], ci[FS];
  auto compute_sg = [&](int half, const XT_& t) {
#pragma unroll
    for (int q = 0; q < SGQ; ++q) {
      const int kl = (half * SGQ + q) * KG;
      if (kbeg + kl < kend) {
        if constexpr (H) {
          hx8 xrh, xrl, xih, xil;
          if constexpr (XC) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float a = t.re[q][e] * sx, b = t.im[q][e] * sx;
              const _Float16 ah = (_Float16)a, bh = (_Float16)b;
              xrh[e] = ah;
              xrl[e] = (_Float16)(a - (float)ah);
              xih[e] = bh;
              xil[e] = (_Float16)(b - (float)bh);
            }
          } else {
            xrh = t.ph[q];
            xrl = t.pl[q];
            xih = xrh;
            xil = xrl;
          }
#pragma unroll
          for (int i = 0; i < FS; ++i) {
            const int row = i * 16 + lr;
            const hx8 srh = *reinterpret_cast<const hx8*>(&sS[0][row][kl + 8 * grp]);
            const hx8 srl = *reinterpret_cast<const hx8*>(&sS[1][row][kl + 8 * grp]);
            hx8 sih = srh, sil = srl;
            if constexpr (SC) {
              sih = *reinterpret_cast<const hx8*>(&sS[NPL - 2][row][kl + 8 * grp]);
              sil = *reinterpret_cast<const hx8*>(&sS[NPL - 1][row][kl + 8 * grp]);
            }
            if constexpr (SA) cmac3<SC, XC>(cr[i], ci[i], srh, srl, sih, sil, xrh, xrl, xih, xil);
            else cmac3<XC, SC>(cr[i], ci[i], xrh, xrl, xih, xil, srh, srl, sih, sil);
          }
        } else {
#pragma unroll
          for (int i = 0; i < FS; ++i) {
            const int row = i * 16 + lr;
            T sr[4], si[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              sr[e] = sS[0][row][kl + 4 * grp + e];
              si[e] = SC ? sS[NPL - 1][row][kl + 4 * grp + e] : T(0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const T xre = t.re[q][e];
              const T xim = XC ? t.im[q][e] : T(0);
              if constexpr (SA) cmac<SC, XC>(cr[i], ci[i], sr[e], si[e], xre, xim);
              else cmac<XC, SC>(cr[i], ci[i], xre, xim, sr[e], si[e]);
            }
          }
        }
      }
    }
  };

  // ---- write one finished tile ----
  // Paired form (float32 output, rows from the shared operand, unit column
  // stride, even row stride and column count, 16-byte aligned output): the
  // lanes of columns 2c and 2c + 1 exchange half of their accumulators (a DPP
  // swap), so that each lane holds two rows of the column pair and writes
  // each row's pair as one 16-byte store: half the store instructions of one
  // 8-byte store per element.  Out-of-range pairs go to the sink, so every
  // tile issues the same 2 FS stores.
  // (used where the streamed operand is real, as in the first contraction)
  constexpr bool PAIRABLE = SA && !XC && std::is_same<OutT, float>::value && std::is_same<T, float>::value;
  typedef float f4v __attribute__((ext_vector_type(4)));
  auto epilogue_pairs = [&](int tx) {
    const int x0 = tx * XT + w * 16;
    const float usc = (float)unscale;                        // a power of two: exact
    const int par = lr & 1;
    const int n0 = x0 + (lr & ~1);
    const bool nv = n0 < xlim;                               // n0 + 1 < xlim as well (xlim even)
    f4v* sink = reinterpret_cast<f4v*>(g.trash) + lane;
#pragma unroll
    for (int i = 0; i < FS; ++i) {
      // DPP quad permutation [1, 0, 3, 2]: exchange with the neighbouring lane
      float sr_[2], si_[2], rr_[2], ri_[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        sr_[j] = par ? cr[i][j] : cr[i][j + 2];
        si_[j] = par ? ci[i][j] : ci[i][j + 2];
        rr_[j] = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sr_[j]), 0xB1, 0xF, 0xF, false));
        ri_[j] = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(si_[j]), 0xB1, 0xF, 0xF, false));
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // rows 4 grp + 2 par + j; columns n0 (lo) and n0 + 1 (hi)
        const int m = s0 + i * 16 + 4 * grp + 2 * par + j;
        const float lre = par ? rr_[j] : cr[i][j], lim = par ? ri_[j] : ci[i][j];
        const float hre = par ? cr[i][2 + j] : rr_[j], him = par ? ci[i][2 + j] : ri_[j];
        f4v v;
        v[0] = lre * usc;
        v[1] = lim * usc;
        v[2] = hre * usc;
        v[3] = him * usc;
        const bool ok = nv && m < slim;
        *opaque(ok ? reinterpret_cast<f4v*>(Cb + 2 * ((i64)m * g.sCm + n0)) : sink) = v;
        if constexpr (H) mx = fmaxf(mx, ok ? fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))) : 0.f);
      }
    }
  };
  auto epilogue = [&](int tx) {
    const int x0 = tx * XT + w * 16;
    const T usc = (T)unscale;                                // a power of two: exact
    // interior tiles (every row and column in range) store without per-element tests
    const bool interior = (x0 + 16 <= xlim) && (s0 + SR <= slim);
    typedef OutT o2 __attribute__((ext_vector_type(2)));
    o2* sink = reinterpret_cast<o2*>(g.trash) + lane;
    if constexpr (SA) {
      const int n = x0 + lr;
      const i64 coff = (i64)n * g.sCn;
      const bool nv = n < g.N;
#pragma unroll
      for (int i = 0; i < FS; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = s0 + i * 16 + frag_row<T>(grp, q);
          const bool ok = interior || (nv && m < g.M);
          o2 v;
          v[0] = (OutT)(cr[i][q] * usc);
          v[1] = (OutT)(ci[i][q] * usc);
          // every element is stored (out-of-range ones into the sink): a fixed
          // number of store instructions per tile
          *opaque(ok ? reinterpret_cast<o2*>(Cb + 2 * (fixoff[q] + i * fixstep + coff)) : sink) = v;
          if constexpr (H) mx = fmaxf(mx, ok ? fmaxf(fabsf((float)v[0]), fabsf((float)v[1])) : 0.f);
        }
      }
    } else {
      i64 roff[4];
      bool rv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = x0 + frag_row<T>(grp, q);
        rv[q] = m < g.M;
        if (g.Mlo > 0) {
          const int mh = m / g.Mlo;
          roff[q] = (i64)mh * g.sCmh + (i64)(m - mh * g.Mlo) * g.sCm;
        } else {
          roff[q] = (i64)m * g.sCm;
        }
      }
#pragma unroll
      for (int i = 0; i < FS; ++i) {
        const int n = s0 + i * 16 + lr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool ok = interior || (rv[q] && n < g.N);
          o2 v;
          v[0] = (OutT)(cr[i][q] * usc);
          v[1] = (OutT)(ci[i][q] * usc);
          *opaque(ok ? reinterpret_cast<o2*>(Cb + 2 * (roff[q] + fixoff[0] + i * fixstep)) : sink) = v;
          if constexpr (H) mx = fmaxf(mx, ok ? fmaxf(fabsf((float)v[0]), fabsf((float)v[1])) : 0.f);
        }
      }
    }
  };

  // super-group 0 of a tile lives in ta, super-group 1 in tb; both loads of
  // the next tile are issued before this tile's stores (the memory counter
  // completes in order, so a load issued after the stores could only be
  // waited for together with them)
  XT_ ta, tb;
  // PAIRS: the paired epilogue (a uniform choice for the whole launch, so each
  // loop issues a fixed sequence of memory operations)
  auto run_tiles = [&](auto PAIRS) {
    constexpr bool P = decltype(PAIRS)::value;
    int tx = pp;
    if (tx < tiles_x) {
      load_sg(tx, 0, ta);
      load_sg(tx, 1, tb);
      // as many sink stores as one tile's epilogue: the loop is entered with
      // the same memory-operation sequence as from its back edge
      if constexpr (P) {
#pragma unroll
        for (int e = 0; e < FS * 2; ++e) *opaque(reinterpret_cast<f4v*>(g.trash) + lane) = f4v{0.f, 0.f, 0.f, 0.f};
      } else {
        typedef OutT o2 __attribute__((ext_vector_type(2)));
        o2 z;
        z[0] = z[1] = (OutT)0;
#pragma unroll
        for (int e = 0; e < FS * 4; ++e) *opaque(reinterpret_cast<o2*>(g.trash) + lane) = z;
      }
    }
    for (; tx < tiles_x; tx += npersist) {
      zero_arr(cr);
      zero_arr(ci);
      const bool more = tx + npersist < tiles_x;
      compute_sg(0, ta);
      if (more) load_sg(tx + npersist, 0, ta);
      compute_sg(1, tb);
      if (more) load_sg(tx + npersist, 1, tb);
      if constexpr (P) epilogue_pairs(tx);
      else epilogue(tx);
    }
  };
  bool pairs = false;
  if constexpr (PAIRABLE)
    pairs = g.sCn == 1 && (g.sCm & 1) == 0 && (xlim & 1) == 0 && (reinterpret_cast<uintptr_t>(Cb) & 15) == 0;
  if (pairs) run_tiles(std::integral_constant<bool, PAIRABLE>{});
  else run_tiles(std::false_type{});
  if constexpr (H) {
    if (g.cmax) {
      mx = wave_max(mx);
      if (lane == 0 && mx > 0.f) atomicMax(g.cmax, __float_as_uint(mx));
    }
  }
}

template <int PK, bool SA, bool SC, bool XC, int FS, int NW, int KS, typename OutT>
__global__ void __launch_bounds__(64 * NW) k_stream1(const StreamArgs g) {
  stream1_body<PK, SA, SC, XC, FS, NW, KS, OutT>(g, blockIdx.x, blockIdx.y, (int)(gridDim.x / g.tiles_m));
}


}  // namespace sb2
