// Second and third contractions of the chain fused into one kernel (split
// float16 arithmetic):
//
//   C[b][j][n][p][r] = sum_s ( sum_q G_b[p][q] A[b][n][j][s][q] ) Gbt_b[r][s]
//
// with Gbt_b[r][s] the transposed reversed-time function (Gbar_b)_sr.  For a
// fixed task (b, n, j) this is the N x N "sandwich" C_bjn = G_b A_bnj^T Gbt_b^T
// of the N x N block A_bnj[s][q]; the middle product Y = A_bnj G_b^T never
// leaves the registers, so the chain's B intermediate is neither written nor
// read back.
//
// Complex products on real matrix cores: the real and imaginary parts share
// the K dimension of one 16x16x32 f16 MFMA.  K slots 8g..8g+7 of lane group
// g = lane/16 hold [x_re(4 indices), x_im(the same 4 indices)], the indices
// being 16c + 4g + 0..3 of a 16-wide chunk c, so that
//   sum over slots of [a_re, a_im] . [b_re, -b_im] = Re sum a b,
//   sum over slots of [a_re, a_im] . [b_im,  b_re] = Im sum a b.
// One MFMA therefore contracts 16 complex indices for one real output part.
//
// Workgroup: NT = ceil(N/16) waves; wave w owns the 16 indices p = 16w..16w+15
// of Y and of C for every task.
//   * G_b[p][:] of the wave's columns: both B operands of step 1, split,
//     kept in registers for the whole slice.
//   * Gbt_b: staged in LDS once per slice b, split, in the slot order above.
//   * A_bnj: streamed through LDS in slabs of 16 rows s (all q), double
//     buffered; each thread loads four consecutive q of one row, splits them
//     and writes them to the free buffer while the other waves still multiply
//     the current one; one barrier per slab.
// Per slab c (s in [16c, 16c + 16)):
//   step 1  Y^T[s][p] = sum_q A[s][q] G[p][q] over the 16-wide q chunks; the
//           accumulators hold rows s = 16c + 4g + i (i = slot 0..3) of column
//           p = lane%16, i.e. exactly the four s indices that lane group g
//           supplies as B operand of
//   step 2  C[p][r] += sum_{s in slab} Y[p][s] Gbt[r][s], with those
//           accumulators as the A operand (a lane supplies row p = lane%16 and
//           the K slots of its group in both operand roles), so C comes out
//           with 16 consecutive r across the lanes of a row.
// Split float16: x 2^e = hi + lo (hi, lo float16, |x 2^e| < 2^14), three MFMAs
// per real product; A, G and Gbt take 2^e from their recorded maxima, Y from
// the bound |Y| <= 2 N max|A| max|G|.  The kernel raises the recorded max |C|
// used by the last contraction.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gemm.hpp"

namespace sb2 {

struct R23Args {
  int N, ns;                 // basis size, slices
  const float* Gs;           // [b][p][q] complex float32
  const float* GbT;          // [b][r][s] complex float32
  const float* A;            // [b][n][j][s][q] complex float32
  float* C;                  // complex float32 (out): [b][j][n][p][r], or [n][b][j][p][r] when chunked
  int chunked;
  const unsigned* gmax;      // recorded max |x| of Gs, GbT, A (float bits)
  const unsigned* gbmax;
  const unsigned* amax;
  unsigned* cmax;            // raised to max |C|
};

// Exponent x of the split scale 2^x for values bounded by m: |v 2^x| < 2^14
// for |v| <= m (x = 0 when m is zero or not finite, reported by `ok`).  `e`
// receives the exponent with m < 2^e.
__device__ __forceinline__ int split_exp(float m, int& e, bool& ok) {
  e = 0;
  ok = m > 0.f && m < 3.0e38f;
  if (!ok) return 0;
  frexpf(m, &e);
  return 14 - e;
}

__device__ __forceinline__ void split_h(float x, _Float16& hi, _Float16& lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (float)hi);
}

template <int NT>
struct R23Cfg {
  static constexpr int NCW = NT;                      // compute waves (one per 16 indices p)
  static constexpr int NTH = 64 * (NT + 1);           // plus one producer wave
  static constexpr int KW = 32 * NT;                  // halves per row: NT chunks x 32 slots
  // row pitch in halves: 16 u bytes with u = 2 mod 4 (KW is a multiple of 32),
  // the pitches for which the 16-byte fragment reads of 16 rows x 4 lane
  // groups are free of LDS bank conflicts on gfx950 (odd u halves the rate)
  static constexpr int LP = KW + 16;
  static constexpr int PI = NT;                       // producer items per lane: 16 ceil(N/4) <= 64 NT
  static_assert(LP >= KW + 8, "row padding holds one 8-slot item");
  static_assert((LP / 8) % 4 == 2, "conflict-free row pitch");
};

// Workgroup wg of nwg: tasks [ntask wg / nwg, ntask (wg + 1) / nwg).
// Waves 0 .. NT-1 compute; wave NT (the producer) streams the A slabs: while
// the compute waves multiply slab g it writes slab g + 1 (loaded two slabs
// earlier) into the free LDS buffer and loads slab g + 3.  The two roles run
// separate loops (their registers do not overlap) with the same barrier
// sequence: one barrier per slab, plus one after staging Gbt when NT = 1.
template <int NT, bool EVEN>
__device__ __forceinline__ void r23_body(const R23Args& a, int wg, int nwg) {
  using C_ = R23Cfg<NT>;
  constexpr int KW = C_::KW, LP = C_::LP, NTH = C_::NTH, PI = C_::PI;
  __shared__ __attribute__((aligned(16))) _Float16 sG[2][16 * NT][LP];   // Gbt slots: hi, lo
  __shared__ __attribute__((aligned(16))) _Float16 sA[2][2][16][LP];     // A slabs: buffer, hi/lo
  __shared__ float red[NT + 1];

  const int N = a.N;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index (uniform)
  const int grp = lane >> 4, lr = lane & 15;
  const i64 nn = (i64)N * N;
  const i64 ntask = (i64)a.ns * nn;
  const i64 t0 = ntask * wg / nwg, t1 = ntask * (wg + 1) / nwg;
  const i64 nslab = (t1 - t0) * NT;                   // slabs of this workgroup, in order
  // scales as exponents, so that no product of scales can overflow
  int ea, eg, egb;
  bool okA, okG, okGb;
  const int xA = split_exp(__uint_as_float(*a.amax), ea, okA);
  const int xG = split_exp(__uint_as_float(*a.gmax), eg, okG);
  const int xGb = split_exp(__uint_as_float(*a.gbmax), egb, okGb);
  const float sGb = ldexpf(1.f, xGb);

  // slots past the last group of four q stay zero for the whole kernel
  const int nc4 = (N + 3) / 4;
  for (int L = tid; L < 2 * 2 * 16 * KW; L += NTH) {
    const int col = L % KW, rest = L / KW;
    if (col >= 8 * nc4) sA[rest / 32][(rest / 16) % 2][rest % 16][col] = (_Float16)0.f;
  }

  // Gbt_b in LDS: row r, slot 32 (s/16) + 8 ((s%16)/4) + (s%4) (+4 for the
  // imaginary part); every wave takes part
  auto stage_gbt = [&](i64 b) {
    const float2* Gb = reinterpret_cast<const float2*>(a.GbT) + b * nn;
    for (int L = tid; L < 16 * NT * 16 * NT; L += NTH) {
      const int r = L / (16 * NT), s = L - r * (16 * NT);
      float2 v = make_float2(0.f, 0.f);
      if (r < N && s < N) v = Gb[(i64)r * N + s];
      const int col = 8 * (s >> 2) + (s & 3);
      split_h(v.x * sGb, sG[0][r][col], sG[1][r][col]);
      split_h(v.y * sGb, sG[0][r][col + 4], sG[1][r][col + 4]);
    }
  };
  // The slab sequence shared by both roles: body(t, b, c, g, buf) for slab g
  // = chunk c of task t, after the barrier that publishes it in buffer buf.
  auto for_slabs = [&](auto&& on_slice, auto&& body) {
    i64 cur_b = -1, g = 0;
#pragma unroll 1
    for (i64 t = t0; t < t1; ++t) {
      const i64 b = t / nn;
#pragma unroll 1
      for (int c = 0; c < NT; ++c, ++g) {             // NT = ceil(N/16) slabs
        __syncthreads();                              // slab g visible; the other buffer free
        if (c == 0 && b != cur_b) {                   // uniform: all waves left the previous slice
          on_slice(b);
          stage_gbt(b);
          cur_b = b;
          if (NT == 1) __syncthreads();               // Gbt is read in this slab already
        }
        body(t, b, c, g, (int)(g & 1));
      }
    }
  };

  if (w == NT) {
    // ---- producer: item u of this lane = row prow[u] of the slab, q = 4 pc4[u] .. + 3
    // (16 ceil(N/4) <= 64 NT items) ----
    const float sAs = ldexpf(1.f, xA);
    // items past 16 ceil(N/4) write zeros into the row padding (never read)
    int prow[PI], pcol[PI], pq[PI];
#pragma unroll
    for (int u = 0; u < PI; ++u) {
      const int L = lane + 64 * u;
      const bool ok = L < 16 * nc4;
      const int r = L / nc4;
      prow[u] = ok ? r : 0;
      pcol[u] = ok ? 8 * (L - r * nc4) : KW;
      pq[u] = ok ? 4 * (L - r * nc4) : 1 << 20;
    }
    // Two register sets: slab x lives in set x % 2 between its load and its
    // store, loaded three slabs ahead of its use, so two slabs are in flight
    // while the compute waves multiply.  Every step issues the same memory
    // operations (loads past the end re-read the last slab and are never
    // stored where a compute wave reads them), so each wait covers only the
    // set being stored.
    float2 pa[PI][4], pb[PI][4];                      // 4 complex per item
    // loads only clamp their addresses (registers untouched until stored, so
    // the loads stay in flight); rows and q past N are zeroed when stored
    auto p_load = [&](i64 g, float2 (&v)[PI][4]) {
      g = g < nslab ? g : nslab - 1;                  // past the end: re-read the last slab
      const i64 t = t0 + g / NT;
      const int c = (int)(g - (g / NT) * NT);
      // uniform base and 32-bit byte offsets (N^2 elements per task)
      const char* base = reinterpret_cast<const char*>(a.A) + (t * nn) * 8;
#pragma unroll
      for (int u = 0; u < PI; ++u) {
        const unsigned ro = (unsigned)(min(16 * c + prow[u], N - 1) * N);
        if constexpr (EVEN) {                         // 16-byte aligned complex pairs (N even)
          const float4 f0 = *reinterpret_cast<const float4*>(base + 8u * (ro + (unsigned)min(pq[u], N - 2)));
          const float4 f1 = *reinterpret_cast<const float4*>(base + 8u * (ro + (unsigned)min(pq[u] + 2, N - 2)));
          v[u][0] = make_float2(f0.x, f0.y);
          v[u][1] = make_float2(f0.z, f0.w);
          v[u][2] = make_float2(f1.x, f1.y);
          v[u][3] = make_float2(f1.z, f1.w);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            v[u][e] = *reinterpret_cast<const float2*>(base + 8u * (ro + (unsigned)min(pq[u] + e, N - 1)));
        }
      }
    };
    // split scale per element: 2^xA inside the block, 0 for q past N (zeroes
    // the element through the product, so that each half of the split is one
    // mixed fused multiply-add)
    float sq[PI][4];
#pragma unroll
    for (int u = 0; u < PI; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) sq[u][e] = pq[u] + e < N ? sAs : 0.f;
    auto p_store_rows = [&](auto all_rows, int c, int buf, const float2 (&v)[PI][4]) {
#pragma unroll
      for (int u = 0; u < PI; ++u) {
        const bool rowok = decltype(all_rows)::value || 16 * c + prow[u] < N;
        float se[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) se[e] = decltype(all_rows)::value ? sq[u][e] : (rowok ? sq[u][e] : 0.f);
        // [re(4), im(4)] as packed pairs
        unsigned h[4], l[4];
        split_pair(v[u][0].x, se[0], v[u][1].x, se[1], h[0], l[0]);
        split_pair(v[u][2].x, se[2], v[u][3].x, se[3], h[1], l[1]);
        split_pair(v[u][0].y, se[0], v[u][1].y, se[1], h[2], l[2]);
        split_pair(v[u][2].y, se[2], v[u][3].y, se[3], h[3], l[3]);
        *reinterpret_cast<ux4*>(&sA[buf][0][prow[u]][pcol[u]]) = ux4{h[0], h[1], h[2], h[3]};
        *reinterpret_cast<ux4*>(&sA[buf][1][prow[u]][pcol[u]]) = ux4{l[0], l[1], l[2], l[3]};
      }
    };
    // slabs inside the block (16 c + 16 <= N) need no row test
    auto p_store = [&](i64 g, int buf, const float2 (&v)[PI][4]) {
      const int c = (int)(g - (g / NT) * NT);
      if (16 * c + 16 <= N) p_store_rows(std::true_type{}, c, buf, v);   // uniform
      else p_store_rows(std::false_type{}, c, buf, v);
    };
    i64 cur_b = -1;
    // one step of the compute waves' barrier sequence: slab g is published,
    // slab g + 1 is written to the free buffer, slab g + 3 is loaded
    auto step = [&](i64 g, float2 (&v)[PI][4]) {
      __syncthreads();
      const i64 t = t0 + g / NT;
      const int c = (int)(g - (g / NT) * NT);
      const i64 b = t / nn;
      if (c == 0 && b != cur_b) {
        stage_gbt(b);
        cur_b = b;
        if (NT == 1) __syncthreads();
      }
      // the producer's stores and loads gate the next slab: they take issue
      // priority over the compute wave that shares its SIMD
      __builtin_amdgcn_s_setprio(2);
      p_store(g + 1, (int)((g + 1) & 1), v);
      p_load(g + 3, v);
      __builtin_amdgcn_s_setprio(0);
    };
    if (nslab > 0) {                                  // slab 0 to buffer 0; slabs 1, 2 in flight
      p_load(0, pa);
      p_store(0, 0, pa);
      p_load(1, pb);
      p_load(2, pa);
      i64 g = 0;
#pragma unroll 1
      for (; g + 1 < nslab; g += 2) {
        step(g, pb);                                  // stores slab g + 1 (odd: set b), loads g + 3
        step(g + 1, pa);                              // stores slab g + 2 (even: set a), loads g + 4
      }
      if (g < nslab) step(g, pb);
    }
    if (lane == 0) red[w] = 0.f;
  } else {
    // ---- compute waves ----
    int nb = 0;                                       // 2 N <= 2^nb
    while ((1 << nb) < 2 * N) ++nb;
    // |Y| <= 2 N max|A| max|G| < 2^(ea + eg + nb)
    const int xY = (okA && okG) ? 14 - (ea + eg + nb) : 0;
    const float sGs = ldexpf(1.f, xG);
    const float fy = ldexpf(1.f, xY - xA - xG);      // accumulator -> Y 2^xY
    const float unscale = ldexpf(1.f, -xGb - xY);
    const int p = 16 * w + lr;                        // this lane's index p in step 1

    // B operands of step 1 for chunk c at q = 16c + 4g + 0..3 of row p, hi
    // and lo: [G_re, -G_im] for the real part and [G_im, G_re] for the
    // imaginary part, both paired with the A fragment [A_re, A_im]
    hx8 bre_h[NT], bre_l[NT], bim_h[NT], bim_l[NT];
    auto load_g = [&](i64 b) {
      const float2* G = reinterpret_cast<const float2*>(a.Gs) + b * nn;
#pragma unroll
      for (int c = 0; c < NT; ++c) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int q = 16 * c + 4 * grp + e;
          float2 v = make_float2(0.f, 0.f);
          if (p < N && q < N) v = G[(i64)p * N + q];
          _Float16 rh, rl, ih, il;
          split_h(v.x * sGs, rh, rl);
          split_h(v.y * sGs, ih, il);
          bre_h[c][e] = rh;
          bre_l[c][e] = rl;
          bre_h[c][4 + e] = -ih;
          bre_l[c][4 + e] = -il;
          bim_h[c][e] = ih;
          bim_l[c][e] = il;
          bim_h[c][4 + e] = rh;
          bim_l[c][4 + e] = rl;
        }
      }
    };

    fx4 cr[NT], ci[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      cr[i] = vzero<fx4>();
      ci[i] = vzero<fx4>();
    }
    float mx = 0.f;
    // B operands of step 2 for the most recent slab: [Y_re, -Y_im] and
    // [Y_im, Y_re] at s = 16c + 4g + i
    hx8 pre_h, pre_l, pim_h, pim_l;
    auto split_y = [&](const fx4& yr, const fx4& yi) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        _Float16 rh, rl, ih, il;
        split_h(yr[i] * fy, rh, rl);
        split_h(yi[i] * fy, ih, il);
        pre_h[i] = rh;
        pre_l[i] = rl;
        pre_h[4 + i] = -ih;
        pre_l[4 + i] = -il;
        pim_h[i] = ih;
        pim_l[i] = il;
        pim_h[4 + i] = rh;
        pim_l[4 + i] = rl;
      }
    };
    // step 2 for slab cs: C[p][r] += Y[p][slab] Gbt[r][slab] with Y as the A
    // operand (lane: row p, the slab's s slots) and Gbt as the B operand
    // (lane: column r), so that the accumulators hold rows p = 16w + 4g + i
    // and 16 consecutive columns r = 16 rt + lane%16
    auto read_g2 = [&](int cs, hx8 (&gh)[NT], hx8 (&gl)[NT]) {
#pragma unroll
      for (int rt = 0; rt < NT; ++rt) {
        const int row = 16 * rt + lr, col = 32 * cs + 8 * grp;
        gh[rt] = *reinterpret_cast<const hx8*>(&sG[0][row][col]);
        gl[rt] = *reinterpret_cast<const hx8*>(&sG[1][row][col]);
      }
    };
    auto step2 = [&](const hx8 (&gh)[NT], const hx8 (&gl)[NT]) {
#pragma unroll
      for (int rt = 0; rt < NT; ++rt) {
        cr[rt] = mma3(pre_h, pre_l, gh[rt], gl[rt], cr[rt]);
        ci[rt] = mma3(pim_h, pim_l, gh[rt], gl[rt], ci[rt]);
      }
    };

    for_slabs(load_g, [&](i64 t, i64 b, int c, i64, int buf) {
      hx8 gh[NT], gl[NT];                             // Gbt fragments of step 2
      __builtin_amdgcn_sched_barrier(0);
      // step 1: Y^T rows 16c .. 16c+15, column p
      fx4 yr = vzero<fx4>(), yi = vzero<fx4>();
      const _Float16* arow = &sA[buf][0][lr][8 * grp];
      constexpr int PL = 16 * LP;                     // hi -> lo plane
      hx8 ah = *reinterpret_cast<const hx8*>(arow), al = *reinterpret_cast<const hx8*>(arow + PL);
#pragma unroll
      for (int qc = 0; qc < NT; ++qc) {
        hx8 nh, nl;                                   // next chunk's fragments, in flight
        if (qc + 1 < NT) {
          nh = *reinterpret_cast<const hx8*>(arow + 32 * (qc + 1));
          nl = *reinterpret_cast<const hx8*>(arow + PL + 32 * (qc + 1));
        }
        yr = mma3(ah, al, bre_h[qc], bre_l[qc], yr);
        yi = mma3(ah, al, bim_h[qc], bim_l[qc], yi);
        if (qc + 1 < NT) {
          ah = nh;
          al = nl;
        }
      }
      // step 2 of the previous slab: its products keep the matrix cores busy
      // while this slab's step-1 results drain and are split; its Gbt
      // fragments are read here rather than ahead of step 1, which keeps
      // fewer registers live
      if (c > 0) {
        read_g2(c - 1, gh, gl);
        step2(gh, gl);
      }
      split_y(yr, yi);
      if (c + 1 < NT) return;
      read_g2(NT - 1, gh, gl);
      step2(gh, gl);
      // ---- store C_bjn[p][r], p = 16 w + 4 g + i, r = 16 rt + lane%16: each
      // store instruction writes 16 consecutive r (128 bytes) of four rows p ----
      const i64 nj = t - b * nn;
      const int n = (int)(nj / N), j = (int)(nj - (i64)(nj / N) * N);
      const i64 blk = a.chunked ? ((i64)n * a.ns + b) * N + j : (b * N + j) * N + n;
      float2* dst = reinterpret_cast<float2*>(a.C) + blk * nn;
#pragma unroll
      for (int rt = 0; rt < NT; ++rt) {
        const int r = 16 * rt + lr;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pp = 16 * w + 4 * grp + i;
          const float re = cr[rt][i] * unscale, im = ci[rt][i] * unscale;
          if (pp < N && r < N) {
            dst[(i64)pp * N + r] = make_float2(re, im);
            mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
          }
        }
        cr[rt] = vzero<fx4>();
        ci[rt] = vzero<fx4>();
      }
    });
    mx = wave_max(mx);
    if (lane == 0) red[w] = mx;
  }
  // block max -> recorded max |C|
  __syncthreads();
  if (tid == 0) {
    float m = 0.f;
#pragma unroll
    for (int i = 0; i <= NT; ++i) m = fmaxf(m, red[i]);
    if (m > 0.f) atomicMax(a.cmax, __float_as_uint(m));
  }
}

template <int NT, bool EVEN>
__global__ void __launch_bounds__(64 * (NT + 1)) k_r23_h16(const R23Args a) {
  r23_body<NT, EVEN>(a, blockIdx.x, gridDim.x);
}

}  // namespace sb2
