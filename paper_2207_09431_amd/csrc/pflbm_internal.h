// pflbm_internal.h -- declarations shared by the kernels and the host runtime
// of the HIP library (not part of the public ABI).
#pragma once

#include "pflbm_device.h"

namespace pflbm {

// fused step kernel variants (pflbm_step.hip)
int step_variant_count();
bool step_variant_shape(int v, int nh, int* tx, int* ty, int* nt);
// state forms of the step: compact float32, stored hbar float32, compact
// float16 (0..2), and the same extended (3..5) with the fixed-point passes of
// the implicit tau, central differences in the hbar forcing, open x ends and
// the link form of the diffusion source
constexpr int kStepForms = 6;
hipError_t launch_step(int v, int nh, int form, const CaseDev* cases, const TileDev* tiles, int ntiles, int par,
                       hipStream_t stream);

// auxiliary kernels (pflbm_aux.hip); `cd_dev` points to the case block in
// device memory, `cd` is the same block on the host (for launch geometry).
// Input fields are float64 planes (ny, nx) in device memory.
hipError_t launch_init(const CaseDev* cd_dev, const CaseDev& cd, int par, const double* C, const double* u,
                       const double* p, hipStream_t stream);
hipError_t launch_macro(const CaseDev* cd_dev, const CaseDev& cd, int par, float* rho, float* u, float* p,
                        float* phi, hipStream_t stream);
hipError_t launch_export(const CaseDev* cd_dev, const CaseDev& cd, int par, float* out, hipStream_t stream);
// scan of one case's state for non-finite values (marks cd.flag)
hipError_t launch_check(const CaseDev* cd_dev, const CaseDev& cd, int par, hipStream_t stream);
// zeroes n non-finite flags
hipError_t launch_clear_flags(unsigned int* flags, int n, hipStream_t stream);
// partial sums of 6 float64 quantities into `partials` (nblocks x 6), then a
// fixed-order final pass into `result` (6 doubles); nblocks = reduce_blocks(cd)
int reduce_blocks(const CaseDev& cd);
hipError_t launch_reduce(const CaseDev* cd_dev, const CaseDev& cd, int par, int comp, double* partials,
                         double* result, hipStream_t stream);

}  // namespace pflbm
