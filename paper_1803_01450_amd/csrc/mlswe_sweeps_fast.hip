// Fast build of the two sweep kernels: the same source with Newton-refined
// hardware reciprocals and reciprocal square roots and floating-point
// contraction (compiled with -ffp-contract=fast).  Results agree with the exact
// build to a few ulps per operation rather than bit for bit.
#define MLSWE_FAST 1
#define MLSWE_NS_VARIANT fast
#include "mlswe_kernels.hpp"
#include "mlswe_wave.hpp"

namespace mlswe {
#define MLSWE_KX k_sweep_x_fast
#define MLSWE_KY k_sweep_y_fast
#define MLSWE_KX1 k_sweep_x1_fast
#define MLSWE_KY1 k_sweep_y1_fast
#define MLSWE_KXR k_sweep_xr_fast
#define MLSWE_KYR k_sweep_yr_fast
#include "mlswe_sweeps.inc"
}  // namespace mlswe
