// General M-layer refine and coarsen (the paper's multilayer formulation for
// any number of layers): launch descriptors and host launchers.
#pragma once
#include <hip/hip_runtime.h>

namespace mlswe {

constexpr int LAYERS_MAX = 8;

// Fine cells of the box (fi0, fj0, fnx, fny) of the fine index space (ratio r)
// refined from a coarse grid of nxc x nyc cells.  Arrays are field-major
// [3M][rows][cols] (h_m, h_m u_m, h_m v_m for layer m = 1 (top) .. M).
struct LayersRefine {
  const double* qc;   // coarse state, [3M][nyc][nxc]
  const double* Bc;   // coarse bathymetry, [nyc][nxc]
  const double* Bf;   // fine bathymetry of the box, [fny][fnx]
  double* qf;         // fine state of the box, [3M][fny][fnx]
  unsigned long long* repairs;  // wet-ordering repairs are added here (nullable)
  long long cplane, fplane;
  int nxc, nyc, r, fi0, fj0, fnx, fny;
  int I0, J0, nI, nJ;  // coarse cells whose children meet the box
  double hdry;
};

// Coarse cells of the box (ci0, cj0, cnx, cny) of a coarse grid (nxc x nyc)
// from their r x r children, given as [3M][r*cny][r*cnx].
struct LayersCoarsen {
  const double* qf;
  double* qc;
  long long cplane, fplane;
  int nxc, r, ci0, cj0, cnx, cny;
  double hdry;
};

// Launch on `stream`; M in 1..LAYERS_MAX.  Return the launch's hipError_t.
hipError_t launch_refine_layers(int M, const LayersRefine& A, hipStream_t stream);
hipError_t launch_coarsen_layers(int M, const LayersCoarsen& A, hipStream_t stream);

}  // namespace mlswe
