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
  static constexpr int NTH = 64 * NT;                 // threads (one wave per 16 columns p)
  static constexpr int KW = 32 * NT;                  // halves per row: NT chunks x 32 slots
  // row pitch in halves, padded so consecutive rows start 16 bytes apart
  // modulo 128 (conflict-free 16-byte fragment reads)
  static constexpr int LP = KW + (((16 - (KW * 2) % 128) + 128) % 128) / 2;
};

// Workgroup wg of nwg: tasks [ntask wg / nwg, ntask (wg + 1) / nwg).
template <int NT>
__device__ __forceinline__ void r23_body(const R23Args& a, int wg, int nwg) {
  using C_ = R23Cfg<NT>;
  constexpr int KW = C_::KW, LP = C_::LP, NTH = C_::NTH;
  __shared__ __attribute__((aligned(16))) _Float16 sG[2][16 * NT][LP];   // Gbt slots: hi, lo
  __shared__ __attribute__((aligned(16))) _Float16 sA[2][2][16][LP];     // A slabs: buffer, hi/lo
  __shared__ float red[NT];

  const int N = a.N;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int grp = lane >> 4, lr = lane & 15;
  const i64 nn = (i64)N * N;
  const i64 ntask = (i64)a.ns * nn;
  const i64 t0 = ntask * wg / nwg, t1 = ntask * (wg + 1) / nwg;
  // scales as exponents, so that no product of scales can overflow
  int ea, eg, egb;
  bool okA, okG, okGb;
  const int xA = split_exp(__uint_as_float(*a.amax), ea, okA);
  const int xG = split_exp(__uint_as_float(*a.gmax), eg, okG);
  const int xGb = split_exp(__uint_as_float(*a.gbmax), egb, okGb);
  int nb = 0;                                         // 2 N <= 2^nb
  while ((1 << nb) < 2 * N) ++nb;
  // |Y| <= 2 N max|A| max|G| < 2^(ea + eg + nb)
  const int xY = (okA && okG) ? 14 - (ea + eg + nb) : 0;
  const float sAs = ldexpf(1.f, xA), sGs = ldexpf(1.f, xG), sGb = ldexpf(1.f, xGb);
  const float fy = ldexpf(1.f, xY - xA - xG);        // accumulator -> Y 2^xY
  const float unscale = ldexpf(1.f, -xGb - xY);
  const int p = 16 * w + lr;                          // this lane's output column

  // slab item of this thread: row srow, q = 4 c4 .. 4 c4 + 3, slots 8 c4 .. 8 c4 + 7
  // (16 ceil(N/4) <= 64 NT items: at most one per thread)
  const int nc4 = (N + 3) / 4;
  const bool has_item = tid < 16 * nc4;
  const int srow = has_item ? tid / nc4 : 0;
  const int c4 = has_item ? tid - srow * nc4 : 0;
  // slots past the last item stay zero for the whole kernel
  for (int L = tid; L < 2 * 2 * 16 * KW; L += NTH) {
    const int col = L % KW, rest = L / KW;
    if (col >= 8 * nc4) sA[rest / 32][(rest / 16) % 2][rest % 16][col] = (_Float16)0.f;
  }

  // branch-free: out-of-range elements read a valid address and are zeroed
  float2 pre[4];
  auto load_slab = [&](i64 t, int c) {
    const int s = 16 * c + srow;
    const bool rowok = has_item && s < N;
    const float2* src = reinterpret_cast<const float2*>(a.A) + t * nn + (rowok ? (i64)s * N + 4 * c4 : 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool ok = rowok && 4 * c4 + e < N;
      const float2 v = src[ok ? e : 0];
      pre[e] = ok ? v : make_float2(0.f, 0.f);
    }
  };
  auto store_slab = [&](int buf) {
    if (!has_item) return;
    hx8 h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      _Float16 x, y;
      split_h(pre[e].x * sAs, x, y);
      h[e] = x;
      l[e] = y;
      split_h(pre[e].y * sAs, x, y);
      h[4 + e] = x;
      l[4 + e] = y;
    }
    *reinterpret_cast<hx8*>(&sA[buf][0][srow][8 * c4]) = h;
    *reinterpret_cast<hx8*>(&sA[buf][1][srow][8 * c4]) = l;
  };

  // ---- per-slice operands ----
  // B operands of step 1 for chunk c: re = [G_re, -G_im], im = [G_im, G_re] at
  // q = 16c + 4g + 0..3 of row p; hi and lo
  hx8 bre_h[NT], bre_l[NT], bim_h[NT], bim_l[NT];
  auto load_slice = [&](i64 b) {
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
    // Gbt_b: row r, slot 32 (s/16) + 8 ((s%16)/4) + (s%4) (+4 for the imaginary part)
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

  fx4 cr[NT], ci[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    cr[i] = vzero<fx4>();
    ci[i] = vzero<fx4>();
  }
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
  // operand (lane: row p, the slab's s slots) and Gbt as the B operand (lane:
  // column r), so that the accumulators hold rows p = 16w + 4g + i and 16
  // consecutive columns r = 16 rt + lane%16
  auto step2 = [&](int cs) {
#pragma unroll
    for (int rt = 0; rt < NT; ++rt) {
      const int row = 16 * rt + lr, col = 32 * cs + 8 * grp;
      const hx8 gh = *reinterpret_cast<const hx8*>(&sG[0][row][col]);
      const hx8 gl = *reinterpret_cast<const hx8*>(&sG[1][row][col]);
      cr[rt] = mma3(pre_h, pre_l, gh, gl, cr[rt]);
      ci[rt] = mma3(pim_h, pim_l, gh, gl, ci[rt]);
    }
  };

  float mx = 0.f;
  i64 cur_b = -1;
  int buf = 0;
  if (t0 < t1) load_slab(t0, 0);

#pragma unroll 1
  for (i64 t = t0; t < t1; ++t) {
    const i64 b = t / nn;
    const i64 nj = t - b * nn;
    const int n = (int)(nj / N), j = (int)(nj - (i64)(nj / N) * N);
    if (b != cur_b) {                                 // uniform across the workgroup
      __syncthreads();                                // every wave is done with the previous Gbt
      load_slice(b);
      cur_b = b;
    }
#pragma unroll 1
    for (int c = 0; c < NT; ++c) {                    // NT = ceil(N/16) slabs
      store_slab(buf);
      {                                               // prefetch the next slab (one call site: one register set)
        const bool last = c + 1 == NT;
        const i64 tn = last ? t + 1 : t;
        if (tn < t1) load_slab(tn, last ? 0 : c + 1);
      }
      __syncthreads();                                // slab c (and Gbt) visible; slab c-1's buffer free

      // step 1: Y^T rows 16c .. 16c+15, column p
      fx4 yr = vzero<fx4>(), yi = vzero<fx4>();
#pragma unroll
      for (int qc = 0; qc < NT; ++qc) {
        const int col = 32 * qc + 8 * grp;
        const hx8 ah = *reinterpret_cast<const hx8*>(&sA[buf][0][lr][col]);
        const hx8 al = *reinterpret_cast<const hx8*>(&sA[buf][1][lr][col]);
        yr = mma3(ah, al, bre_h[qc], bre_l[qc], yr);
        yi = mma3(ah, al, bim_h[qc], bim_l[qc], yi);
      }
      // step 2 of the previous slab: its products keep the matrix cores busy
      // while this slab's step-1 results drain and are split
      if (c > 0) step2(c - 1);
      split_y(yr, yi);
      buf ^= 1;
    }
    step2(NT - 1);

    // ---- store C_bjn[p][r], p = 16 w + 4 g + i, r = 16 rt + lane%16: each
    // store instruction writes 16 consecutive r (128 bytes) of four rows p ----
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
  }
  // block max -> recorded max |C|
  mx = wave_max(mx);
  if (lane == 0) red[w] = mx;
  __syncthreads();
  if (tid == 0) {
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < NT; ++i) m = fmaxf(m, red[i]);
    if (m > 0.f) atomicMax(a.cmax, __float_as_uint(m));
  }
}

template <int NT>
__global__ void __launch_bounds__(64 * NT) k_r23_h16(const R23Args a) {
  r23_body<NT>(a, blockIdx.x, gridDim.x);
}

}  // namespace sb2
