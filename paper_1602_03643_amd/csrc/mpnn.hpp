// Internal interface of the learned warm start (the network is defined in
// mpnn.hip; the C ABI entry points are declared in oasis.h).
#pragma once

#include "oasis.h"

namespace oasis {

// The forward pass of oasis_mpnn_forward for inference inside a step:
// writes the guess phi_prev + sigma * delta only; the activations a
// backward pass would need are not kept in ws.
int mpnn_infer(void *stream, const oasis_csr *Ks, const double *s, int32_t dim, const double *coords,
               const double *b_phi, const double *phi_prev, const float *params, double *guess, void *ws,
               size_t ws_bytes);

}  // namespace oasis
