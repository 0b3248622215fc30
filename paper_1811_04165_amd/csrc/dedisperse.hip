// Brute-force dedispersion on gfx950.
//
//   dd[i][t] = sum over c of in[c][t + delay[i][c]]
//
// A work-group owns a tile of `dpb` consecutive DM trials by `tpd * spt`
// consecutive output samples.  It walks the channels `cu` at a time: the
// group stages, for each of those channels, the input window every DM of the
// tile needs (it starts at the first DM's delay; later DMs read further in,
// never by more than (dpb - 1) * max_step samples) into LDS, widened from
// uint8 to 16 bits, in two copies shifted by one sample so that every DM can
// read sample pairs as aligned dwords.  Each wavefront owns one DM trial and
// 64 * spt samples; lane l accumulates sample pairs (2l + 128k, 2l + 128k + 1)
// as two 16-bit lanes of one dword (a packed SWAR add: one dword read and one
// add per two samples), flushing into 32-bit totals every 256 channels
// (256 * 255 < 2^16).  The delay of the wave's DM for a channel is uniform
// across the wave, so its LDS address is a scalar plus the lane offset.
#include "internal.h"

namespace amber {
namespace {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// v_perm_b32 selectors: bytes of {hi:next, lo:cur}; 0x0c yields a zero byte.
constexpr uint32_t kSel01 = 0x0c010c00u;  // [0 b1 0 b0]  samples 0,1
constexpr uint32_t kSel23 = 0x0c030c02u;  // [0 b3 0 b2]  samples 2,3
constexpr uint32_t kSel12 = 0x0c020c01u;  // [0 b2 0 b1]  samples 1,2
constexpr uint32_t kSel34 = 0x0c040c03u;  // [0 b4 0 b3]  samples 3,4 (b4 = next dword's b0)

template <int SPT, int CU>
__global__ __launch_bounds__(1024) void dedisperse_kernel(
    const int32_t *__restrict__ delays, int n_dm, int n_chan,
    const uint8_t *__restrict__ in, int64_t in_stride, int64_t in_bytes,
    int32_t *__restrict__ dd, int64_t dd_stride, int64_t n_out,
    int tpd, int dpb, int win, int omax, int store_pairs)
{
    constexpr int M = SPT / 2;  // sample pairs (dwords) per lane
    extern __shared__ uint4 lds4[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);

    const int win2 = win >> 1;        // dwords per staged row copy
    const int items_per_row = win >> 4;  // staging items of 16 samples
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int wave = uniform(tid >> 6);
    const int lane = tid & 63;
    const int waves_per_dm = tpd >> 6;
    const int dm_local = uniform(wave / waves_per_dm);
    const int wave_t = uniform((wave - dm_local * waves_per_dm) * 64 * SPT);
    const int i0 = blockIdx.y * dpb;
    const int i = i0 + dm_local;
    const bool active = i < n_dm;
    const int64_t t0 = (int64_t)blockIdx.x * tpd * SPT;

    const int32_t *__restrict__ dfirst = delays + (size_t)i0 * n_chan;
    const int32_t *__restrict__ dmine = delays + (size_t)(active ? i : i0) * n_chan;
    const int n_items = CU * items_per_row;

    uint32_t acc[M];
    uint32_t lo[M], hi[M];
#pragma unroll
    for (int k = 0; k < M; ++k) acc[k] = lo[k] = hi[k] = 0u;

    int since_flush = 0;
    for (int c0 = 0; c0 < n_chan; c0 += CU) {
        // ---- stage CU channel windows into LDS (two 16-bit copies) ----
        for (int q = tid; q < n_items; q += nthreads) {
            const int j = q / items_per_row;
            const int it = q - j * items_per_row;
            const int c = c0 + j;
            uint32_t w[5] = {0u, 0u, 0u, 0u, 0u};
            if (c < n_chan) {
                const int64_t start = t0 + dfirst[c];
                const int64_t g0 = start & ~(int64_t)3;
                const int64_t off = (int64_t)c * in_stride + g0 + 16 * (int64_t)it;
                if (off >= 0 && off + 20 <= in_bytes) {
                    const uint32_t *src = reinterpret_cast<const uint32_t *>(in + off);
#pragma unroll
                    for (int k = 0; k < 5; ++k) w[k] = src[k];
                } else {
                    // only dwords outside the buffer are replaced (by zero): they lie
                    // past the last row's samples, so no output < n_out reads them
                    const uint32_t *src = reinterpret_cast<const uint32_t *>(in);
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        const int64_t o = off + 4 * k;
                        w[k] = (o >= 0 && o + 4 <= in_bytes) ? src[o >> 2] : 0u;
                    }
                }
            }
            uint4 *r0 = lds4 + ((j * win2) >> 2) + it * 2;
            uint4 *r1 = lds4 + (((CU + j) * win2) >> 2) + it * 2;
            uint4 a, b, e, f;
            a.x = __builtin_amdgcn_perm(w[1], w[0], kSel01); a.y = __builtin_amdgcn_perm(w[1], w[0], kSel23);
            a.z = __builtin_amdgcn_perm(w[2], w[1], kSel01); a.w = __builtin_amdgcn_perm(w[2], w[1], kSel23);
            b.x = __builtin_amdgcn_perm(w[3], w[2], kSel01); b.y = __builtin_amdgcn_perm(w[3], w[2], kSel23);
            b.z = __builtin_amdgcn_perm(w[4], w[3], kSel01); b.w = __builtin_amdgcn_perm(w[4], w[3], kSel23);
            e.x = __builtin_amdgcn_perm(w[1], w[0], kSel12); e.y = __builtin_amdgcn_perm(w[1], w[0], kSel34);
            e.z = __builtin_amdgcn_perm(w[2], w[1], kSel12); e.w = __builtin_amdgcn_perm(w[2], w[1], kSel34);
            f.x = __builtin_amdgcn_perm(w[3], w[2], kSel12); f.y = __builtin_amdgcn_perm(w[3], w[2], kSel34);
            f.z = __builtin_amdgcn_perm(w[4], w[3], kSel12); f.w = __builtin_amdgcn_perm(w[4], w[3], kSel34);
            r0[0] = a; r0[1] = b;
            r1[0] = e; r1[1] = f;
        }
        __syncthreads();

        // ---- accumulate: one dword read + one packed add per sample pair ----
        if (active) {
#pragma unroll
            for (int j = 0; j < CU; ++j) {
                const int c = c0 + j;
                if (c < n_chan) {
                    const int df = dfirst[c];
                    const int d = dmine[c];
                    const int lead = df & 3;
                    int o = d - df + lead;
                    o = o < 0 ? 0 : (o > omax ? omax : o);
                    const int row = (o & 1) ? (CU + j) : j;
                    const uint32_t *src = lds + row * win2 + (o >> 1) + (wave_t >> 1) + lane;
#pragma unroll
                    for (int k = 0; k < M; ++k) acc[k] += src[64 * k];
                }
            }
            since_flush += CU;
            if (since_flush >= 256) {
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    lo[k] += acc[k] & 0xffffu;
                    hi[k] += acc[k] >> 16;
                    acc[k] = 0u;
                }
                since_flush = 0;
            }
        }
        __syncthreads();
    }

    if (!active) return;
    int32_t *__restrict__ out = dd + (size_t)i * dd_stride;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int64_t t = t0 + wave_t + 128 * k + 2 * lane;
        const int32_t v0 = (int32_t)(lo[k] + (acc[k] & 0xffffu));
        const int32_t v1 = (int32_t)(hi[k] + (acc[k] >> 16));
        if (t + 1 < n_out && store_pairs) {
            *reinterpret_cast<int2 *>(out + t) = make_int2(v0, v1);
        } else {
            if (t < n_out) out[t] = v0;
            if (t + 1 < n_out) out[t + 1] = v1;
        }
    }
}

using KernelFn = void (*)(const int32_t *, int, int, const uint8_t *, int64_t, int64_t, int32_t *, int64_t, int64_t,
                          int, int, int, int, int);

template <int SPT>
KernelFn pick_cu(int cu)
{
    switch (cu) {
    case 1: return dedisperse_kernel<SPT, 1>;
    case 2: return dedisperse_kernel<SPT, 2>;
    case 4: return dedisperse_kernel<SPT, 4>;
    case 8: return dedisperse_kernel<SPT, 8>;
    case 16: return dedisperse_kernel<SPT, 16>;
    }
    return nullptr;
}

KernelFn pick(int spt, int cu)
{
    switch (spt) {
    case 2: return pick_cu<2>(cu);
    case 4: return pick_cu<4>(cu);
    case 8: return pick_cu<8>(cu);
    case 16: return pick_cu<16>(cu);
    }
    return nullptr;
}

}  // namespace

amber_status launch_dedisperse(const DedispPlan &p, const int32_t *d_delays, int n_dm, int n_chan,
                               const uint8_t *d_in, int64_t in_stride, int64_t n_in, int32_t *d_dd,
                               int64_t dd_stride, int64_t n_out, hipStream_t stream)
{
    (void)n_in;
    KernelFn fn = pick(p.spt, p.cu);
    if (!fn) return fail(AMBER_E_CONFIG, "no dedispersion kernel for spt=%d cu=%d", p.spt, p.cu);
    if (p.lds_bytes > 64 * 1024)
        AMBER_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes),
                  "hipFuncSetAttribute(dedisperse)");
    const int64_t tiles_t = (n_out + p.tile_t - 1) / p.tile_t;
    const int64_t tiles_dm = (n_dm + p.dpb - 1) / p.dpb;
    if (tiles_t > 0x7fffffff || tiles_dm > 65535)
        return fail(AMBER_E_SHAPE, "grid of %lld x %lld tiles is too large", (long long)tiles_t, (long long)tiles_dm);
    const int store_pairs = (dd_stride % 2 == 0) && (((uintptr_t)d_dd & 7) == 0);
    dim3 grid((unsigned)tiles_t, (unsigned)tiles_dm);
    hipLaunchKernelGGL(fn, grid, dim3(p.threads), (size_t)p.lds_bytes, stream, d_delays, n_dm, n_chan, d_in,
                       in_stride, (int64_t)n_chan * in_stride, d_dd, dd_stride, n_out, p.tpd, p.dpb, p.win, p.omax,
                       store_pairs);
    AMBER_HIP(hipGetLastError(), "dedisperse launch");
    return AMBER_OK;
}

}  // namespace amber
