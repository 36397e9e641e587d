// Streaming device copy (qds_stream_copy in include/qds.h): the read + write
// bandwidth ceiling the marched kernels are compared with.  16 bytes per lane,
// a grid-stride loop over a fixed grid, optionally with the non-temporal
// (streaming) hint on loads and stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qds.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_cu32x4;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

template <bool NT>
__global__ void __launch_bounds__(256) k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n) {
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride) {
        if constexpr (NT) {
            const u32x4 v = __builtin_nontemporal_load((g_cu32x4*)(src + q));
            __builtin_nontemporal_store(v, (g_u32x4*)(dst + q));
        } else {
            *(g_u32x4*)(dst + q) = *(g_cu32x4*)(src + q);
        }
    }
}

}  // namespace

extern "C" qds_status qds_stream_copy(void* dst, const void* src, size_t bytes, int32_t streaming, int32_t blocks,
                                      void* stream) {
    if (!dst || !src || bytes % 16 != 0 || blocks < 1) return QDS_EINVAL;
    const size_t n = bytes / 16;
    if (n == 0) return QDS_OK;
    const dim3 grd{unsigned(blocks), 1, 1};
    const dim3 blk{256, 1, 1};
    if (streaming)
        hipLaunchKernelGGL(k_copy16<true>, grd, blk, 0, hipStream_t(stream), static_cast<const u32x4*>(src),
                           static_cast<u32x4*>(dst), n);
    else
        hipLaunchKernelGGL(k_copy16<false>, grd, blk, 0, hipStream_t(stream), static_cast<const u32x4*>(src),
                           static_cast<u32x4*>(dst), n);
    return hipGetLastError() == hipSuccess ? QDS_OK : QDS_EHIP;
}
