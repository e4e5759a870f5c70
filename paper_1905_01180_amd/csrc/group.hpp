// Split-float16 contraction chain on the n-chunked layout, for one system's
// chunk (argument builders shared by the single-system launches) and for
// several systems in one launch: the fused second+third contraction and the
// last contraction of every member whose basis size falls in the same 16-wide
// bucket (the kernels are specialised on ceil(N/16)) run as one grid; member
// i owns the workgroups [off[i], off[i+1]) and reads its chunk description
// from the device table of chain refs.
#pragma once
#include "chain.hpp"
#include "r4.hpp"
#include "sandwich.hpp"

namespace sb2 {

// Fused second+third contraction: A in X1 -> C in X2 (n-chunked).
__host__ __device__ inline R23Args r23_args(const ChainRefs& r) {
  R23Args a;
  a.N = r.N;
  a.ns = r.ns;
  a.Gs = reinterpret_cast<const float*>(r.Gs);
  a.GbT = reinterpret_cast<const float*>(r.GbT);
  a.A = reinterpret_cast<const float*>(r.X1);
  a.C = reinterpret_cast<float*>(r.X2);
  a.gmax = r.scal + S_GMAX;
  a.gbmax = r.scal + S_GBMAX;
  a.amax = r.scal + S_AMAX;
  a.cmax = r.scal + S_CMAX;
  a.chunked = r.chunked;
  return a;
}

// Last contraction on the n-chunked layout: C in X2 (or C3), one chunk per n.
__host__ __device__ inline R4Args r4_args(const ChainRefs& r) {
  R4Args a;
  a.M = r.N;
  a.ncol = r.ns * r.N;
  a.kc = r.N * r.N;
  a.V = reinterpret_cast<const _Float16*>(r.Vp);
  a.ldv = r.KpV;
  a.vplane = (i64)r.N * r.KpV;
  a.vchunk = r.KB;
  a.X = reinterpret_cast<const float*>(r.C3 ? r.C3 : r.X2);
  a.xchunk = (i64)a.ncol * a.kc;
  a.part = reinterpret_cast<double*>(r.part);
  a.vmax = r.scal + S_VMAX;
  a.xmax = r.scal + S_CMAX;
  return a;
}

// Members of one bucket: refs index and workgroup range of each.
struct SubGroup {
  int count;
  int idx[MAX_GROUP];
  long long off[MAX_GROUP + 1];
};

__device__ __forceinline__ int sub_member(const SubGroup& t, long long b) {
  int i = 0;
  while (i + 1 < t.count && b >= t.off[i + 1]) ++i;
  return i;
}

template <int NT>
__global__ void __launch_bounds__(64 * (NT + 1)) k_r23_group(const ChainRefs* __restrict__ refs, const SubGroup t) {
  const long long b = blockIdx.x;
  const int i = sub_member(t, b);
  const R23Args a = r23_args(refs[t.idx[i]]);
  r23_body<NT, false>(a, (int)(b - t.off[i]), (int)(t.off[i + 1] - t.off[i]));   // members of any parity
}

template <int FS>
__global__ void __launch_bounds__(R4_THREADS) k_r4_group(const ChainRefs* __restrict__ refs, const SubGroup t) {
  const long long b = blockIdx.x;
  const int i = sub_member(t, b);
  const R4Args a = r4_args(refs[t.idx[i]]);
  const int tiles = r4_tiles(a);
  const int local = (int)(b - t.off[i]);
  r4_body<FS, false>(a, local % tiles, local / tiles);   // 8-byte pair loads: any chunk length
}

}  // namespace sb2
