// The FP32 product of the kernel matrix (v_mfma_f32_32x32x2f32), one 128 x 128
// tile per workgroup, in a translation unit of its own so that the library's
// sources compile in parallel.
#include "gram_tile.h"

namespace kkm {
namespace gt {

namespace {

template <typename OUT, bool FULL>
__global__ __launch_bounds__(GTHREADS, 2) void gram_f32_mfma(F32Tile a, TileOrder o) {
    __shared__ __attribute__((aligned(16))) F32Lds lds;
    int64_t bi, bj;
    if (!tile_of_block(o, bi, bj)) return;
    f32_tile<OUT, FULL>(a, bi, bj, lds);
}

}  // namespace

void launch_gram_f32(int32_t k_store, bool full, dim3 g, const F32Tile &a, const TileOrder &order,
                     hipStream_t stream) {
    const dim3 b(GTHREADS);
    if (k_store == KKM_F32 && !full)
        hipLaunchKernelGGL((gram_f32_mfma<float, false>), g, b, 0, stream, a, order);
    else if (k_store == KKM_F32)
        hipLaunchKernelGGL((gram_f32_mfma<float, true>), g, b, 0, stream, a, order);
    else if (!full)
        hipLaunchKernelGGL((gram_f32_mfma<uint16_t, false>), g, b, 0, stream, a, order);
    else
        hipLaunchKernelGGL((gram_f32_mfma<uint16_t, true>), g, b, 0, stream, a, order);
}

}  // namespace gt
}  // namespace kkm
