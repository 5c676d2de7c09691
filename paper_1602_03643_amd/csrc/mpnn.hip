// Learned warm start (message-passing network): placeholder entry points
// until the kernels land.
#include "internal.hpp"

extern "C" int oasis_mpnn_workspace_size(int32_t, size_t *) { return OASIS_EUNSUPPORTED; }
extern "C" int oasis_mpnn_forward(void *, const oasis_csr *, const double *, int32_t, const double *,
                                  const double *, const double *, const float *, double *, float *, void *,
                                  size_t) {
    return OASIS_EUNSUPPORTED;
}
extern "C" int oasis_mpnn_backward(void *, const oasis_csr *, const double *, const double *, const double *,
                                   const float *, float *, double *, void *, size_t) {
    return OASIS_EUNSUPPORTED;
}
extern "C" int oasis_mpnn_adam(void *, float *, const float *, float *, float *, int32_t, float, float, float,
                               float) {
    return OASIS_EUNSUPPORTED;
}
