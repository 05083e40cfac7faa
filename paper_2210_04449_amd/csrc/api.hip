// Status strings, version and the device error word.
#include <algorithm>

#include "common.hpp"

extern "C" const char *rtsdf_status_string(int status)
{
    switch (status) {
    case RTSDF_OK: return "ok";
    case RTSDF_EINVAL: return "invalid argument";
    case RTSDF_ENOMEM: return "out of device memory";
    case RTSDF_EHIP: return "HIP runtime error";
    case RTSDF_EDEVICE: return "device-side error reported";
    default: return "unknown status";
    }
}

extern "C" int rtsdf_version(void) { return 100; }

extern "C" int rtsdf_sync_status(rtsdf_stream stream, uint32_t *bits)
{
    using namespace rtsdf;
    if (hipStreamSynchronize(as_stream(stream)) != hipSuccess) return RTSDF_EHIP;
    unsigned int word = 0, zero = 0;
    if (hipMemcpyFromSymbol(&word, HIP_SYMBOL(g_error_word), sizeof(word), 0, hipMemcpyDeviceToHost) != hipSuccess)
        return RTSDF_EHIP;
    if (word != 0 &&
        hipMemcpyToSymbol(HIP_SYMBOL(g_error_word), &zero, sizeof(zero), 0, hipMemcpyHostToDevice) != hipSuccess)
        return RTSDF_EHIP;
    if (bits) *bits = word;
    return word ? RTSDF_EDEVICE : RTSDF_OK;
}

extern "C" int rtsdf_copy(void *dst, const void *src, size_t bytes, rtsdf_stream stream)
{
    if (bytes == 0) return RTSDF_OK;
    if (!dst || !src) return RTSDF_EINVAL;
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, rtsdf::as_stream(stream)) != hipSuccess)
        return RTSDF_EHIP;
    return RTSDF_OK;
}

namespace rtsdf {

// The library's square root, one value per lane (grid-stride).
__global__ void __launch_bounds__(256) sqrt_kernel(const float *__restrict__ x, int64_t n, float *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) out[i] = rn_sqrt(x[i]);
}

}  // namespace rtsdf

extern "C" int rtsdf_sqrt(const float *x, int64_t n, float *out, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (n < 0 || (n > 0 && (!x || !out))) return RTSDF_EINVAL;
    if (n == 0) return RTSDF_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)num_cus() * 64);
    sqrt_kernel<<<dim3((unsigned)blocks), dim3(256), 0, as_stream(stream)>>>(x, n, out);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}
