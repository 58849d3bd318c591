// gsn_corrector_internal.hpp -- hooks between the grid solver and the learned
// corrector (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "gsn.h"

// psi <- psi + s_out * net(Re psi, Im psi, phi) for one image, queued on s.
gsn_status corrector_correct_inplace(gsn_corrector c, float2 *psi, const float *phi, hipStream_t s);
int corrector_height(gsn_corrector c);
int corrector_width(gsn_corrector c);
// device scratch of the corrector for one image: phi (float), two psi copies
float *corrector_phi_buffer(gsn_corrector c);
float2 *corrector_psi_buffer(gsn_corrector c, int which);
