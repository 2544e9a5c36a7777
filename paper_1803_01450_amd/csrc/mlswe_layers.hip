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
// For even r the children move in 16-byte pairs (loads for coarsen, stores
// for refine) where the layout allows it.
#include <hip/hip_runtime.h>

#include "mlswe_layers.hpp"

namespace mlswe {
namespace {

__device__ __forceinline__ double minmod2(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

// Per-layer interpolation data of one coarse cell (register arrays).
template <int M>
struct LayerSlopes {
  double e[M], sex[M], sey[M], u[M], sux[M], suy[M], v[M], svx[M], svy[M];
  bool wc[M];
};

// Depths of one child at fractions (fa, fb) over fine bathymetry Bf: from the
// bottom layer up through the effective bathymetry, thin ones dry, then the
// wet ordering (repairs counted).
template <int M>
__device__ __forceinline__ void child_depths(const LayerSlopes<M>& S, double fa, double fb, double Bf, double hdry,
                                             double h[M], unsigned& rep) {
  double Bhat = Bf;
#pragma unroll
  for (int m = M - 1; m >= 0; --m) {
    const double ef = (S.e[m] + S.sex[m] * fa) + S.sey[m] * fb;
    double hm = S.wc[m] ? ef - Bhat : 0.0;
    if (hm < hdry) hm = 0.0;
    h[m] = hm;
    Bhat = Bhat + hm;
  }
  bool dry_above = false;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (dry_above && h[m] > 0.0) { h[m] = 0.0; ++rep; }
    if (h[m] == 0.0) dry_above = true;
  }
}

// Momenta of layer m of a child: the limited interpolant where the fine layer
// is wet, else zero.
template <int M>
__device__ __forceinline__ double mom_u(const LayerSlopes<M>& S, int m, double fa, double fb, double h) {
  return h > 0.0 ? (S.u[m] + S.sux[m] * fa) + S.suy[m] * fb : 0.0;
}
template <int M>
__device__ __forceinline__ double mom_v(const LayerSlopes<M>& S, int m, double fa, double fb, double h) {
  return h > 0.0 ? (S.v[m] + S.svx[m] * fa) + S.svy[m] * fb : 0.0;
}

// PAIRS: r even and every pair of children (a, a + 1), a even, lies on a
// 16-byte boundary of the fine box (even box origin and width, 16-byte aligned
// arrays): each pair is written with one 16-byte store per field, so the
// lanes of a wave fill a contiguous span of the fine row with each store.
template <int M, bool PAIRS>
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
    LayerSlopes<M> S;
    double s0 = A.Bc[k0], sl = A.Bc[kl], sr = A.Bc[kr], sd = A.Bc[kd], su = A.Bc[ku];
#pragma unroll
    for (int m = M - 1; m >= 0; --m) {  // layer m + 1, bottom layer first
      const double* h = A.qc + 3 * m * A.cplane;
      const double h0 = h[k0], hl = h[kl], hr = h[kr], hd = h[kd], hu = h[ku];
      s0 = s0 + h0; sl = sl + hl; sr = sr + hr; sd = sd + hd; su = su + hu;
      const bool w0 = h0 >= A.hdry;
      const bool okx = inx && hl >= A.hdry && w0 && hr >= A.hdry;
      const bool oky = iny && hd >= A.hdry && w0 && hu >= A.hdry;
      S.wc[m] = w0;
      S.e[m] = s0;
      S.sex[m] = okx ? minmod2(s0 - sl, sr - s0) : 0.0;
      S.sey[m] = oky ? minmod2(s0 - sd, su - s0) : 0.0;
      const double* pu = h + A.cplane;
      const double u0 = pu[k0];
      S.u[m] = u0;
      S.sux[m] = okx ? minmod2(u0 - pu[kl], pu[kr] - u0) : 0.0;
      S.suy[m] = oky ? minmod2(u0 - pu[kd], pu[ku] - u0) : 0.0;
      const double* pv = pu + A.cplane;
      const double v0 = pv[k0];
      S.v[m] = v0;
      S.svx[m] = okx ? minmod2(v0 - pv[kl], pv[kr] - v0) : 0.0;
      S.svy[m] = oky ? minmod2(v0 - pv[kd], pv[ku] - v0) : 0.0;
    }
    const int r = A.r;
    for (int b = 0; b < r; ++b) {
      const int fj = r * J + b - A.fj0;
      if (fj < 0 || fj >= A.fny) continue;
      const double fb = double(2 * b + 1 - r) / double(2 * r);
      if (PAIRS) {
        for (int a = 0; a < r; a += 2) {
          const int fi = r * I + a - A.fi0;  // even; the pair lies wholly inside or outside the box
          if (fi < 0 || fi >= A.fnx) continue;
          const double fa0 = double(2 * a + 1 - r) / double(2 * r);
          const double fa1 = double(2 * a + 3 - r) / double(2 * r);
          const long long kf = (long long)fj * A.fnx + fi;
          const double2 B2 = *reinterpret_cast<const double2*>(A.Bf + kf);
          double h0[M], h1[M];
          child_depths<M>(S, fa0, fb, B2.x, A.hdry, h0, rep);
          child_depths<M>(S, fa1, fb, B2.y, A.hdry, h1, rep);
#pragma unroll
          for (int m = 0; m < M; ++m) {
            double* o = A.qf + 3 * m * A.fplane + kf;
            *reinterpret_cast<double2*>(o) = make_double2(h0[m], h1[m]);
            *reinterpret_cast<double2*>(o + A.fplane) =
                make_double2(mom_u<M>(S, m, fa0, fb, h0[m]), mom_u<M>(S, m, fa1, fb, h1[m]));
            *reinterpret_cast<double2*>(o + 2 * A.fplane) =
                make_double2(mom_v<M>(S, m, fa0, fb, h0[m]), mom_v<M>(S, m, fa1, fb, h1[m]));
          }
        }
      } else {
        for (int a = 0; a < r; ++a) {
          const int fi = r * I + a - A.fi0;
          if (fi < 0 || fi >= A.fnx) continue;
          const double fa = double(2 * a + 1 - r) / double(2 * r);
          const long long kf = (long long)fj * A.fnx + fi;
          double h[M];
          child_depths<M>(S, fa, fb, A.Bf[kf], A.hdry, h, rep);
#pragma unroll
          for (int m = 0; m < M; ++m) {
            double* o = A.qf + 3 * m * A.fplane + kf;
            o[0] = h[m];
            o[A.fplane] = mom_u<M>(S, m, fa, fb, h[m]);
            o[2 * A.fplane] = mom_v<M>(S, m, fa, fb, h[m]);
          }
        }
      }
    }
  }
  if (A.repairs) {
    for (int o = 32; o > 0; o >>= 1) rep += __shfl_xor(rep, o, 64);
    if ((threadIdx.x & 63) == 0 && rep) atomicAdd(A.repairs, (unsigned long long)rep);
  }
}

// PAIRS: r even and a 16-byte aligned fine array: children read two at a time
// (16-byte loads, contiguous across the lanes), summed in the same order.
template <int M, bool PAIRS>
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
    for (int bb = 0; bb < r; ++bb) {
      if (PAIRS) {
        for (int aa = 0; aa < r; aa += 2) {
          const double2 v = *reinterpret_cast<const double2*>(p + bb * fnx + aa);
          s = s + v.x;
          s = s + v.y;
        }
      } else {
        for (int aa = 0; aa < r; ++aa) s = s + p[bb * fnx + aa];
      }
    }
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
  const dim3 grid((A.nI + 63) / 64, (A.nJ + 3) / 4);
  const bool pairs = A.r % 2 == 0 && A.fi0 % 2 == 0 && A.fnx % 2 == 0 &&
                     (reinterpret_cast<uintptr_t>(A.qf) & 15) == 0 && (reinterpret_cast<uintptr_t>(A.Bf) & 15) == 0;
  if (pairs)
    hipLaunchKernelGGL((k_refine_layers<M, true>), grid, dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL((k_refine_layers<M, false>), grid, dim3(256), 0, s, A);
  return hipGetLastError();
}

template <int M>
hipError_t coarsen_m(const LayersCoarsen& A, hipStream_t s) {
  const dim3 grid((A.cnx + 63) / 64, (A.cny + 3) / 4);
  if (A.r % 2 == 0 && (reinterpret_cast<uintptr_t>(A.qf) & 15) == 0)
    hipLaunchKernelGGL((k_coarsen_layers<M, true>), grid, dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL((k_coarsen_layers<M, false>), grid, dim3(256), 0, s, A);
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
