// The BF16 / FP8 product of the kernel matrix (v_mfma_f32_32x32x16_bf16 /
// _fp8_fp8, FP32 accumulation), 128 x 128 tiles three workgroups per CU, and
// the selectable 256 x 256 tile.  A translation unit of its own so that the
// library's sources compile in parallel.
#include "gram_tile.h"

namespace kkm {
namespace gt {

namespace {

// One tile per workgroup, three workgroups per CU (single-buffered slabs).
template <int PREC, typename OUT, bool FULL>
__global__ __launch_bounds__(GTHREADS, 3) void gram_lowp_mfma(LowpTile a, TileOrder o) {
    __shared__ __attribute__((aligned(16))) LowpLds<false> lds;
    int64_t bi, bj;
    if (!tile_of_block(o, bi, bj)) return;
    lowp_tile<PREC, OUT, FULL, false>(a, bi, bj, lds);
}

template <bool FULL>
void lowp_dispatch(int32_t gram_prec, int32_t k_store, dim3 g, dim3 b, const LowpTile &a,
                   const TileOrder &order, hipStream_t stream) {
    if (gram_prec == KKM_BF16 && k_store == KKM_F32)
        hipLaunchKernelGGL((gram_lowp_mfma<KKM_BF16, float, FULL>), g, b, 0, stream, a, order);
    else if (gram_prec == KKM_BF16)
        hipLaunchKernelGGL((gram_lowp_mfma<KKM_BF16, uint16_t, FULL>), g, b, 0, stream, a, order);
    else if (k_store == KKM_F32)
        hipLaunchKernelGGL((gram_lowp_mfma<KKM_FP8_ROWSCALED, float, FULL>), g, b, 0, stream, a,
                           order);
    else
        hipLaunchKernelGGL((gram_lowp_mfma<KKM_FP8_ROWSCALED, uint16_t, FULL>), g, b, 0, stream,
                           a, order);
}

}  // namespace

void launch_gram_lowp(int32_t gram_prec, int32_t k_store, bool full, dim3 g, const LowpTile &a,
                      const TileOrder &order, hipStream_t stream) {
    if (full)
        lowp_dispatch<true>(gram_prec, k_store, g, dim3(GTHREADS), a, order, stream);
    else
        lowp_dispatch<false>(gram_prec, k_store, g, dim3(GTHREADS), a, order, stream);
}

}  // namespace gt
}  // namespace kkm
