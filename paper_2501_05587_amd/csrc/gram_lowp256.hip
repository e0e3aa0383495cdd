// The selectable 256 x 256 tile of the BF16 / FP8 product (one workgroup per
// CU), in a translation unit of its own so that the library's sources compile
// in parallel.
#include "gram_tile.h"

namespace kkm {
namespace gt {

namespace {

template <int PREC, typename OUT>
__global__ __launch_bounds__(GTHREADS, 1) void gram_lowp_mfma256(LowpTile a, TileOrder o) {
    __shared__ __attribute__((aligned(16))) LowpLds256 lds;
    int64_t bi, bj;
    if (!tile_of_block(o, bi, bj)) return;
    lowp_tile256<PREC, OUT>(a, bi, bj, lds);
}

}  // namespace

void launch_gram_lowp256(int32_t gram_prec, int32_t k_store, dim3 g, const LowpTile &a,
                         const TileOrder &order, hipStream_t stream) {
    const dim3 b(GTHREADS);
    if (gram_prec == KKM_BF16 && k_store == KKM_F32)
        hipLaunchKernelGGL((gram_lowp_mfma256<KKM_BF16, float>), g, b, 0, stream, a, order);
    else if (gram_prec == KKM_BF16)
        hipLaunchKernelGGL((gram_lowp_mfma256<KKM_BF16, uint16_t>), g, b, 0, stream, a, order);
    else if (k_store == KKM_F32)
        hipLaunchKernelGGL((gram_lowp_mfma256<KKM_FP8_ROWSCALED, float>), g, b, 0, stream, a, order);
    else
        hipLaunchKernelGGL((gram_lowp_mfma256<KKM_FP8_ROWSCALED, uint16_t>), g, b, 0, stream, a,
                           order);
}

}  // namespace gt
}  // namespace kkm
