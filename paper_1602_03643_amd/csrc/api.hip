// Error reporting and version of the C ABI.
#include "internal.hpp"

namespace oasis {
static thread_local int g_last_hip_error = 0;
void set_hip_error(hipError_t e) { g_last_hip_error = static_cast<int>(e); }
}  // namespace oasis

extern "C" const char *oasis_strerror(int code) {
    switch (code) {
        case OASIS_OK: return "ok";
        case OASIS_EINVAL: return "invalid argument";
        case OASIS_EHIP: return "HIP runtime error";
        case OASIS_ENOTCONV: return "Krylov solver did not converge within maxit";
        case OASIS_EBREAKDOWN: return "Krylov solver breakdown";
        case OASIS_ENAN: return "non-finite value in a reduction";
        case OASIS_EWORKSPACE: return "workspace too small";
        case OASIS_EUNSUPPORTED: return "input outside a documented limit";
        default: return "unknown error";
    }
}

extern "C" int oasis_last_hip_error(void) { return oasis::g_last_hip_error; }

extern "C" const char *oasis_version(void) { return "oasis-mi355x 0.1 (gfx950)"; }
