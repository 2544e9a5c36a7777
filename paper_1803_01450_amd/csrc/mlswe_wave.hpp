// Lane exchange, wave reductions and level-array indexing shared by the HIP
// kernels (both builds of the sweeps include it).
#pragma once
#include "mlswe_kernels.hpp"

namespace mlswe {
inline namespace MLSWE_NS_VARIANT {

__device__ __forceinline__ long long cidx(long long pitch, int i, int j) {
  return (long long)(j + 2) * pitch + (long long)(i + XOFF);
}

// Row access in the sweeps: a wave-uniform base (field plane and row, kept in
// scalar registers) plus the lane's 32-bit byte offset within the row, which
// is the scalar-base form of the global loads and stores.  Offsets stay far
// below 2^32: a row holds at most a few thousand columns.
// The level arrays are device allocations, so the accesses are issued as
// global (not flat) memory operations.
typedef __attribute__((address_space(1))) const char gchar_c;
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ unsigned lane_boff(int i) { return (unsigned)(i + XOFF) * 8u; }
__device__ __forceinline__ gchar_c* row_of(const double* a, long long off) { return (gchar_c*)(a + off); }
__device__ __forceinline__ double ld_at(gchar_c* row, unsigned boff) {
  return *(__attribute__((address_space(1))) const double*)(row + boff);
}
// Coverage byte: wave-uniform row offset plus the lane's column offset.
__device__ __forceinline__ int ld_cov(const unsigned char* m, long long rowoff, unsigned col) {
  return *((__attribute__((address_space(1))) const unsigned char*)(m + rowoff) + col);
}
__device__ __forceinline__ void st_at(double* a, long long off, unsigned boff, double v) {
  *(__attribute__((address_space(1))) double*)((gchar*)(a + off) + boff) = v;
}

// Whole-wave rotations by one lane through DPP (wave_ror:1 / wave_rol:1): every
// lane receives a value, so no copy of the old register is needed.  The end
// lanes receive the other end's value; they are halo lanes whose edges feed no
// update, speed or counter.
__device__ __forceinline__ int dpp_up_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_dn_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xf, 0xf, false); }
__device__ __forceinline__ double shup(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_up_i((int)(unsigned)b), hi = (unsigned)dpp_up_i((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double shdn(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_dn_i((int)(unsigned)b), hi = (unsigned)dpp_dn_i((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ int shup_i(int v) { return dpp_up_i(v); }

// The surfaces and wet flags are formed again from the moved depths and
// bathymetry, by the same expressions as load_cell (cheaper than moving them).
__device__ __forceinline__ CellX shup_cell(const PhysParams& P, const CellX& c) {
  CellX o;
  o.h1 = shup(c.h1); o.m1 = shup(c.m1); o.t1 = shup(c.t1);
  o.h2 = shup(c.h2); o.m2 = shup(c.m2); o.t2 = shup(c.t2); o.B = shup(c.B);
  o.u1 = shup(c.u1); o.w1 = shup(c.w1); o.u2 = shup(c.u2); o.w2 = shup(c.w2);
  o.s1 = shup(c.s1); o.s2 = shup(c.s2);
  o.e2 = o.B + o.h2;
  o.e1 = o.e2 + o.h1;
  o.wet1 = o.h1 >= P.hdry;
  o.wet2 = o.h2 >= P.hdry;
  return o;
}

__device__ __forceinline__ EdgeW shup_edge(const EdgeW& w) {
  EdgeW o;
#pragma unroll
  for (int p = 0; p < 6; ++p) o.s[p] = shup(w.s[p]);
#pragma unroll
  for (int p = 0; p < 4; ++p) { o.A[p] = shup(w.A[p]); o.C[p] = shup(w.C[p]); }
  o.v1 = shup(w.v1); o.v2 = shup(w.v2); o.z4 = shup(w.z4); o.z5 = shup(w.z5);
  int m = shup_i(w.mode1 | (w.mode2 << 4));
  o.mode1 = m & 15; o.mode2 = m >> 4;
  return o;
}

__device__ __forceinline__ int shdn_i(int v) { return dpp_dn_i(v); }

__device__ __forceinline__ EdgeW shdn_edge(const EdgeW& w) {
  EdgeW o;
#pragma unroll
  for (int p = 0; p < 6; ++p) o.s[p] = shdn(w.s[p]);
#pragma unroll
  for (int p = 0; p < 4; ++p) { o.A[p] = shdn(w.A[p]); o.C[p] = shdn(w.C[p]); }
  o.v1 = shdn(w.v1); o.v2 = shdn(w.v2); o.z4 = shdn(w.z4); o.z5 = shdn(w.z5);
  int m = shdn_i(w.mode1 | (w.mode2 << 4));
  o.mode1 = m & 15; o.mode2 = m >> 4;
  return o;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) { double t = __shfl_xor(v, o, 64); v = t > v ? t : v; }
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void flush_part(TilePart* part, double smax, int hyp, const FixCount& K, int lane) {
  const double sm = wave_max(smax);
  const int h = wave_isum(hyp);
  const int nc = wave_isum(K.nclip);
  const int rp = wave_isum(K.repair);
  const int nf = wave_isum(K.nonfinite);
  const double c1 = wave_sum(K.clip1);
  const double c2 = wave_sum(K.clip2);
  if (lane == 0) {
    part->smax = sm;
    part->clip1 = c1;
    part->clip2 = c2;
    part->hyp = (unsigned)h;
    part->nclip = (unsigned)nc;
    part->repair = (unsigned)rp;
    part->nonfinite = nf != 0 ? 1u : 0u;
  }
}

// Branch code of wave p's limiter and speed sign at an edge, weighted by a hash
// of the edge position; sums of these over a run change (almost surely) when any
// limiter branch or wave direction changes.
__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ unsigned long long branch_sig(const EdgeW& W, const double dd[6], const double dl[6],
                                                         const double dr[6], int i, int j, int axis) {
  unsigned long long acc = 0;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    const double sv = W.s[p];
    unsigned code = sv > 0.0 ? 1u : (sv < 0.0 ? 2u : 3u);
    if (slot_mode(W, p) == 0 && sv != 0.0 && dd[p] != 0.0) {
      const double th = (sv > 0.0 ? dl[p] : dr[p]) / dd[p];
      const double a = 0.5 * (1.0 + th), b = 2.0 * th;
      const double m1 = a < 2.0 ? a : 2.0;
      const double m = m1 < b ? m1 : b;
      unsigned br = (0.0 > m) ? 1u : (m1 < b ? (a < 2.0 ? 2u : 3u) : 4u);
      code |= br << 2;
    }
    const unsigned long long key =
        ((unsigned long long)(unsigned)i << 32) ^ ((unsigned long long)(unsigned)j << 4) ^ (unsigned)(axis * 8 + p);
    acc += (unsigned long long)code * mix64(key);
  }
  return acc;
}

__device__ __forceinline__ unsigned long long wave_usum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double edge_smax(const EdgeW& W) {
  double m = 0.0;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    double a = W.s[p] < 0.0 ? 0.0 - W.s[p] : W.s[p];
    if (a > m) m = a;
  }
  return m;
}

}  // inline namespace
}  // namespace mlswe
