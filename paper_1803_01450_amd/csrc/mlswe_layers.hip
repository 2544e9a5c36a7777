// General M-layer refine and coarsen (Sec. 2.1, Eqs. 4-5 and 10; Sec. 2.2,
// Eq. 11), for M = 1 .. LAYERS_MAX layers of one grid, FP64.
//
// Refine: one lane per coarse cell.  The lane loads the five-point stencil of
// every field once, forms each layer's surface from the bathymetry upwards
// (eta_M = B + h_M, eta_m = eta_{m+1} + h_m), its minmod slopes and those of
// the layer's momenta, then writes all r x r children: fine surface
// (eta + sx fa) + sy fb with fa = (2a + 1 - r) / (2r), depths from the bottom
// layer up through the effective bathymetry (fine bathymetry plus the fine
// layers below), thin depths dry, then every layer below a dry one dry
// (counted), momenta by the same limited interpolant where the fine layer is
// wet.  Slopes are zero across the domain edge and for a layer dry in any of
// the three cells of a direction; a dry coarse layer refines to a dry layer.
// Lanes of a wave take consecutive coarse cells of a row, so the r stores of a
// child row of a field together fill one contiguous span of the fine row.
//
// Coarsen: one lane per coarse cell; the row-major sum of its children times
// 1/r^2 for every field, then the same fix-up (thin layers dry, wet ordering).
#include <hip/hip_runtime.h>

#include "mlswe_layers.hpp"

namespace mlswe {
namespace {

__device__ __forceinline__ double minmod2(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

template <int M>
__global__ __launch_bounds__(256) void k_refine_layers(LayersRefine A) {
  const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
  const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
  unsigned rep = 0;
  if (gx < A.nI && gy < A.nJ) {
    const int I = A.I0 + gx, J = A.J0 + gy;
    const bool inx = I - 1 >= 0 && I + 1 < A.nxc;
    const bool iny = J - 1 >= 0 && J + 1 < A.nyc;
    const long long k0 = (long long)J * A.nxc + I;
    // an absent neighbour reads the centre; its slope is then zero anyway
    const long long kl = inx ? k0 - 1 : k0, kr = inx ? k0 + 1 : k0;
    const long long kd = iny ? k0 - A.nxc : k0, ku = iny ? k0 + A.nxc : k0;
    double e[M], sex[M], sey[M], u[M], sux[M], suy[M], v[M], svx[M], svy[M];
    bool wc[M];
    double s0 = A.Bc[k0], sl = A.Bc[kl], sr = A.Bc[kr], sd = A.Bc[kd], su = A.Bc[ku];
#pragma unroll
    for (int m = M - 1; m >= 0; --m) {  // layer m + 1, bottom layer first
      const double* h = A.qc + 3 * m * A.cplane;
      const double h0 = h[k0], hl = h[kl], hr = h[kr], hd = h[kd], hu = h[ku];
      s0 = s0 + h0; sl = sl + hl; sr = sr + hr; sd = sd + hd; su = su + hu;
      const bool w0 = h0 >= A.hdry;
      const bool okx = inx && hl >= A.hdry && w0 && hr >= A.hdry;
      const bool oky = iny && hd >= A.hdry && w0 && hu >= A.hdry;
      wc[m] = w0;
      e[m] = s0;
      sex[m] = okx ? minmod2(s0 - sl, sr - s0) : 0.0;
      sey[m] = oky ? minmod2(s0 - sd, su - s0) : 0.0;
      const double* pu = h + A.cplane;
      const double u0 = pu[k0];
      u[m] = u0;
      sux[m] = okx ? minmod2(u0 - pu[kl], pu[kr] - u0) : 0.0;
      suy[m] = oky ? minmod2(u0 - pu[kd], pu[ku] - u0) : 0.0;
      const double* pv = pu + A.cplane;
      const double v0 = pv[k0];
      v[m] = v0;
      svx[m] = okx ? minmod2(v0 - pv[kl], pv[kr] - v0) : 0.0;
      svy[m] = oky ? minmod2(v0 - pv[kd], pv[ku] - v0) : 0.0;
    }
    const int r = A.r;
    for (int b = 0; b < r; ++b) {
      const int fj = r * J + b - A.fj0;
      if (fj < 0 || fj >= A.fny) continue;
      const double fb = double(2 * b + 1 - r) / double(2 * r);
      for (int a = 0; a < r; ++a) {
        const int fi = r * I + a - A.fi0;
        if (fi < 0 || fi >= A.fnx) continue;
        const double fa = double(2 * a + 1 - r) / double(2 * r);
        const long long kf = (long long)fj * A.fnx + fi;
        double h[M];
        double Bhat = A.Bf[kf];
#pragma unroll
        for (int m = M - 1; m >= 0; --m) {
          const double ef = (e[m] + sex[m] * fa) + sey[m] * fb;
          double hm = wc[m] ? ef - Bhat : 0.0;
          if (hm < A.hdry) hm = 0.0;
          h[m] = hm;
          Bhat = Bhat + hm;
        }
        bool dry_above = false;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (dry_above && h[m] > 0.0) { h[m] = 0.0; ++rep; }
          if (h[m] == 0.0) dry_above = true;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
          double* o = A.qf + 3 * m * A.fplane + kf;
          const bool wet = h[m] > 0.0;
          o[0] = h[m];
          o[A.fplane] = wet ? (u[m] + sux[m] * fa) + suy[m] * fb : 0.0;
          o[2 * A.fplane] = wet ? (v[m] + svx[m] * fa) + svy[m] * fb : 0.0;
        }
      }
    }
  }
  if (A.repairs) {
    for (int o = 32; o > 0; o >>= 1) rep += __shfl_xor(rep, o, 64);
    if ((threadIdx.x & 63) == 0 && rep) atomicAdd(A.repairs, (unsigned long long)rep);
  }
}

template <int M>
__global__ __launch_bounds__(256) void k_coarsen_layers(LayersCoarsen A) {
  const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
  const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (gx >= A.cnx || gy >= A.cny) return;
  const int r = A.r;
  const long long fnx = (long long)r * A.cnx;
  const double inv = 1.0 / double(r * r);
  double q[3 * M];
#pragma unroll
  for (int f = 0; f < 3 * M; ++f) {
    const double* p = A.qf + f * A.fplane + (long long)r * gy * fnx + (long long)r * gx;
    double s = 0.0;
    for (int bb = 0; bb < r; ++bb)
      for (int aa = 0; aa < r; ++aa) s = s + p[bb * fnx + aa];
    q[f] = s * inv;
  }
#pragma unroll
  for (int m = M - 1; m >= 0; --m)
    if (q[3 * m] < A.hdry) { q[3 * m] = 0.0; q[3 * m + 1] = 0.0; q[3 * m + 2] = 0.0; }
  bool dry_above = false;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (dry_above && q[3 * m] > 0.0) { q[3 * m] = 0.0; q[3 * m + 1] = 0.0; q[3 * m + 2] = 0.0; }
    if (q[3 * m] == 0.0) dry_above = true;
  }
  const long long kc = (long long)(A.cj0 + gy) * A.nxc + (A.ci0 + gx);
#pragma unroll
  for (int f = 0; f < 3 * M; ++f) A.qc[f * A.cplane + kc] = q[f];
}

template <int M>
hipError_t refine_m(const LayersRefine& A, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_layers<M>, dim3((A.nI + 63) / 64, (A.nJ + 3) / 4), dim3(256), 0, s, A);
  return hipGetLastError();
}

template <int M>
hipError_t coarsen_m(const LayersCoarsen& A, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen_layers<M>, dim3((A.cnx + 63) / 64, (A.cny + 3) / 4), dim3(256), 0, s, A);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_refine_layers(int M, const LayersRefine& A, hipStream_t s) {
  switch (M) {
    case 1: return refine_m<1>(A, s);
    case 2: return refine_m<2>(A, s);
    case 3: return refine_m<3>(A, s);
    case 4: return refine_m<4>(A, s);
    case 5: return refine_m<5>(A, s);
    case 6: return refine_m<6>(A, s);
    case 7: return refine_m<7>(A, s);
    case 8: return refine_m<8>(A, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_coarsen_layers(int M, const LayersCoarsen& A, hipStream_t s) {
  switch (M) {
    case 1: return coarsen_m<1>(A, s);
    case 2: return coarsen_m<2>(A, s);
    case 3: return coarsen_m<3>(A, s);
    case 4: return coarsen_m<4>(A, s);
    case 5: return coarsen_m<5>(A, s);
    case 6: return coarsen_m<6>(A, s);
    case 7: return coarsen_m<7>(A, s);
    case 8: return coarsen_m<8>(A, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mlswe
