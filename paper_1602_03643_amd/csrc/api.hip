// Error reporting and version of the C ABI.
#include "internal.hpp"

#include <cstring>

namespace oasis {
static thread_local int g_last_hip_error = 0;
void set_hip_error(hipError_t e) { g_last_hip_error = static_cast<int>(e); }

__global__ __launch_bounds__(kBlock) void k_publish(const unsigned *__restrict__ src, unsigned *__restrict__ dst,
                                                    int words) {
    for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}

void stage_alloc(HostStage &st) {
    st = HostStage{};
    void *h = nullptr, *d = nullptr;
    if (hipHostMalloc(&h, kStageBytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return;
    }
    st.h = h;
    st.d = d;
}

void stage_free(HostStage &st) {
    if (st.h) (void)hipHostFree(st.h);
    st = HostStage{};
}

int read_state(hipStream_t s, const HostStage &st, const void *dev, void *out, size_t bytes) {
    if (st.h && bytes <= kStageBytes && bytes % 4 == 0) {
        hipLaunchKernelGGL(k_publish, dim3(1), dim3(kBlock), 0, s, static_cast<const unsigned *>(dev),
                           static_cast<unsigned *>(st.d), static_cast<int>(bytes / 4));
        OASIS_TRY_LAUNCH();
        OASIS_TRY_HIP(hipStreamSynchronize(s));
        std::memcpy(out, st.h, bytes);
        return OASIS_OK;
    }
    OASIS_TRY_HIP(hipMemcpyAsync(out, dev, bytes, hipMemcpyDeviceToHost, s));
    OASIS_TRY_HIP(hipStreamSynchronize(s));
    return OASIS_OK;
}

int write_state(hipStream_t s, const HostStage &st, void *dev, const void *src, size_t bytes) {
    if (st.h && bytes <= kStageBytes && bytes % 4 == 0) {
        std::memcpy(st.h, src, bytes);
        hipLaunchKernelGGL(k_publish, dim3(1), dim3(kBlock), 0, s, static_cast<const unsigned *>(st.d),
                           static_cast<unsigned *>(dev), static_cast<int>(bytes / 4));
        OASIS_TRY_LAUNCH();
        return OASIS_OK;
    }
    OASIS_TRY_HIP(hipMemcpyAsync(dev, src, bytes, hipMemcpyHostToDevice, s));
    return OASIS_OK;
}
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
