// gsn_corrector_internal.hpp -- hooks between the grid solver and the learned
// corrector (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "gsn.h"

// One image, queued on s: with u = e^{i theta} psi the state as the caller
// reads it (theta: the grid's FP64 global phase, a device scalar),
// psi <- psi + s_out e^{-i theta} net(Re u, Im u, phi).
gsn_status corrector_correct_inplace(gsn_corrector c, float2 *psi, const float *phi, const double *theta,
                                     hipStream_t s);
int corrector_height(gsn_corrector c);
int corrector_width(gsn_corrector c);
// device scratch of the corrector for one image: phi (float), two psi copies
float *corrector_phi_buffer(gsn_corrector c);
float2 *corrector_psi_buffer(gsn_corrector c, int which);
