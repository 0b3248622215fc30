// Input window of one streamed chunk.
//
// A beam streamed in chunks of L samples keeps windows of D + L samples per
// channel (D = its largest delay).  Row c of the chunk's window holds the last
// D samples of the previous window, prev[c][L, L + D), followed by the
// chunk's own samples, staged contiguously as stage[c][0, L).  One pass over
// the window writes both parts, so a chunk needs one contiguous host-to-device
// copy and one launch instead of two strided copies.
#include "internal.h"

namespace amber {
namespace {

__global__ __launch_bounds__(256) void assemble_kernel(uint8_t *__restrict__ cur, const uint8_t *__restrict__ prev,
                                                       const uint8_t *__restrict__ stage, int64_t stride, int64_t L,
                                                       int64_t D)
{
    const int64_t c = blockIdx.y;
    const int64_t p = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);  // first byte of this dword
    const int64_t row = D + L;
    if (p >= row) return;
    const uint8_t *pr = prev + c * stride + L;
    const uint8_t *st = stage + c * L;
    uint32_t v = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t q = p + j;
        const uint32_t b = q < D ? pr[q] : (q < row ? st[q - D] : 0u);
        v |= b << (8 * j);
    }
    // rows are padded to a multiple of 4 bytes, so the dword stays in the row
    *reinterpret_cast<uint32_t *>(cur + c * stride + p) = v;
}

}  // namespace

amber_status launch_assemble(uint8_t *d_cur, const uint8_t *d_prev, const uint8_t *d_stage, int n_chan,
                             int64_t stride, int64_t L, int64_t D, hipStream_t stream)
{
    if (n_chan < 1 || L < 1 || D < 0 || stride < D + L || stride % 4 != 0 || ((uintptr_t)d_cur & 3) != 0)
        return fail(AMBER_E_ARG, "bad window geometry for chunk assembly");
    const int64_t dwords = (D + L + 3) / 4;
    const int64_t bx = (dwords + 255) / 256;
    if (bx > 0x7fffffff || n_chan > 65535) return fail(AMBER_E_SHAPE, "chunk window too large to assemble");
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)bx, (unsigned)n_chan), dim3(256), 0, stream, d_cur, d_prev,
                       d_stage, stride, L, D);
    AMBER_HIP(hipGetLastError(), "assemble launch");
    return AMBER_OK;
}

}  // namespace amber
