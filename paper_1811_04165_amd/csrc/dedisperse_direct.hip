// Brute-force dedispersion that reads its input straight from global memory
// through the caches, with no staging in LDS (the paper's localMem gene set
// to off; the staged kernel is the gene's other value).
//
//   dd[i][t] = sum over c of in[c][t + delay[i][c]]
//
// Work decomposition as in the staged kernel: a work-group owns dpb
// consecutive DM trials and tpd * spt consecutive output samples, each
// wavefront one DM trial and 64 * spt samples.  Here lane l owns the spt
// consecutive samples t_l = t_wave + l * spt, so the wave's reads of one
// channel are one contiguous span and coalesce.
//
// Per channel a lane loads the spt / 4 + 1 aligned dwords that hold
// in[c][t_l + delay .. t_l + delay + spt).  t_l is a multiple of 4, so the
// byte misalignment s = delay mod 4 is the same on every lane, and one
// wave-uniform v_perm_b32 selector both realigns and widens: output dword k
// takes bytes s + 4k and s + 4k + 2 of the dword pair {k + 1, k}, zero-
// extended into two 16-bit halves, and a second selector takes s + 4k + 1
// and s + 4k + 3.  Each 32-bit add then advances two running sums; after at
// most 256 channels the halves are added into 32-bit totals.  A zapped
// channel (keep flag 0), or a channel past the end of a partial group, gets
// the all-zero selector and adds nothing.
#include "internal.h"

namespace amber {
namespace {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *global(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}

// v_perm_b32 selector: bytes a and a + 2 of {hi, lo} into the low byte of
// each 16-bit half (0x0c selects a zero byte).
__device__ __forceinline__ uint32_t pair_sel(uint32_t a)
{
    return a | 0x0c00u | ((a + 2u) << 16) | 0x0c000000u;
}

constexpr uint32_t kZeroSel = 0x0c0c0c0cu;

template <int SPT, int CU>
__global__ __launch_bounds__(1024) void dedisperse_direct_kernel(DedispJob single, const DedispJob *__restrict__ jobs,
                                                                 int n_jobs, int tpd, int dpb)
{
    constexpr int K = SPT / 4;  // output dwords per lane
    constexpr int W = K + 1;    // input dwords loaded per lane and channel

    int block = blockIdx.x;
    DedispJob job = single;
    if (jobs) {
        int j = 0;
        while (j + 1 < n_jobs && jobs[j + 1].block_start <= block) ++j;
        job = jobs[j];
        block -= job.block_start;
    }
    const int n_dm = job.n_dm, n_chan = job.n_chan;
    const int64_t n_out = job.n_out;
    const int tx = block % job.tiles_t, ty = block / job.tiles_t;

    const int tid = threadIdx.x;
    const int wave = uniform(tid >> 6);
    const int lane = tid & 63;
    const int waves_per_dm = tpd >> 6;
    const int dm_local = uniform(wave / waves_per_dm);
    const int i = ty * dpb + dm_local;
    if (i >= n_dm) return;  // no barriers below: a wave past the last DM leaves
    const int64_t t_wave = (int64_t)tx * tpd * SPT + (int64_t)(wave - dm_local * waves_per_dm) * 64 * SPT;
    const int64_t t_l = t_wave + (int64_t)lane * SPT;

    const int32_t *__restrict__ drow = job.delays + (size_t)i * n_chan;
    const uint8_t *__restrict__ keep = job.keep;
    const int64_t row_dwords = job.in_stride >> 2;  // the stride is a multiple of 4

    uint32_t tot[SPT], lo[K], hi[K];
#pragma unroll
    for (int k = 0; k < SPT; ++k) tot[k] = 0u;
#pragma unroll
    for (int k = 0; k < K; ++k) lo[k] = hi[k] = 0u;

    for (int c0 = 0; c0 < n_chan; c0 += 64) {
        // lane j holds the delay and keep flag of channel c0 + j
        const int cj = c0 + lane;
        const int dj = cj < n_chan ? *global(drow + cj) : 0;
        const int kj = cj < n_chan ? (keep ? (int)*global(keep + cj) : 1) : 0;
        const int nc = n_chan - c0 < 64 ? n_chan - c0 : 64;
        for (int cc = 0; cc < nc; cc += CU) {
            uint32_t d[CU][W];
            uint32_t sl[CU], sh[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                int off = __builtin_amdgcn_readlane(dj, cc + u);
                off = off < 0 ? 0 : off;  // table entries are >= 0; a bad one cannot read before the row
                const int kp = __builtin_amdgcn_readlane(kj, cc + u);
                int c = c0 + cc + u;
                c = c < n_chan ? c : n_chan - 1;  // past the end: a valid row, zero selector
                const uint32_t *row = reinterpret_cast<const uint32_t *>(job.in + (size_t)c * job.in_stride);
                const int64_t b = (t_l + off) >> 2;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const int64_t idx = b + w < row_dwords ? b + w : row_dwords - 1;
                    d[u][w] = *global(row + idx);
                }
                const uint32_t s = (uint32_t)off & 3u;
                sl[u] = kp ? pair_sel(s) : kZeroSel;
                sh[u] = kp ? pair_sel(s + 1u) : kZeroSel;
            }
#pragma unroll
            for (int u = 0; u < CU; ++u)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    lo[k] += __builtin_amdgcn_perm(d[u][k + 1], d[u][k], sl[u]);
                    hi[k] += __builtin_amdgcn_perm(d[u][k + 1], d[u][k], sh[u]);
                }
        }
        // at most 256 channels since the last widening (c0 is a multiple of 64)
        if (((c0 + 64) & 255) == 0 || c0 + 64 >= n_chan) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                tot[4 * k + 0] += lo[k] & 0xffffu;
                tot[4 * k + 2] += lo[k] >> 16;
                tot[4 * k + 1] += hi[k] & 0xffffu;
                tot[4 * k + 3] += hi[k] >> 16;
                lo[k] = hi[k] = 0u;
            }
        }
    }

    int32_t *out = job.dd + (size_t)i * job.dd_stride;
    if (t_l + SPT <= n_out && ((reinterpret_cast<uintptr_t>(out + t_l) & 15) == 0)) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int k = 0; k < K; ++k) {
            u32x4 v = {tot[4 * k], tot[4 * k + 1], tot[4 * k + 2], tot[4 * k + 3]};
            *reinterpret_cast<u32x4 *>(out + t_l + 4 * k) = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SPT; ++k)
            if (t_l + k < n_out) out[t_l + k] = (int32_t)tot[k];
    }
}

using DirectFn = void (*)(DedispJob, const DedispJob *, int, int, int);

template <int SPT>
DirectFn pick_cu(int cu)
{
    // loaded dwords per lane, (SPT / 4 + 1) * CU, stay within 64 registers
    switch (cu) {
    case 1: return dedisperse_direct_kernel<SPT, 1>;
    case 2: return dedisperse_direct_kernel<SPT, 2>;
    case 4: return dedisperse_direct_kernel<SPT, 4>;
    case 8:
        if constexpr ((SPT / 4 + 1) * 8 <= 64) return dedisperse_direct_kernel<SPT, 8>;
        return nullptr;
    case 16:
        if constexpr ((SPT / 4 + 1) * 16 <= 64) return dedisperse_direct_kernel<SPT, 16>;
        return nullptr;
    case 32:
        if constexpr ((SPT / 4 + 1) * 32 <= 64) return dedisperse_direct_kernel<SPT, 32>;
        return nullptr;
    }
    return nullptr;
}

DirectFn pick(int spt, int cu)
{
    switch (spt) {
    case 4: return pick_cu<4>(cu);
    case 8: return pick_cu<8>(cu);
    case 16: return pick_cu<16>(cu);
    case 32: return pick_cu<32>(cu);
    }
    return nullptr;
}

}  // namespace

amber_status launch_dedisperse_direct_jobs(const DedispPlan &p, const DedispJob *single, const DedispJob *d_jobs,
                                           int n_jobs, int64_t n_blocks, hipStream_t stream)
{
    DirectFn fn = pick(p.spt, p.cu);
    if (!fn)
        return fail(AMBER_E_CONFIG, "no direct-read dedispersion kernel for spt=%d cu=%d", p.spt, p.cu);
    if (single && (single->groups > 1 || single->in_u16 || single->out_u16))
        return fail(AMBER_E_CONFIG, "direct reads take one uint8 problem with int32 sums");
    if (n_blocks > 0x7fffffff) return fail(AMBER_E_SHAPE, "grid of %lld work-groups is too large", (long long)n_blocks);
    hipLaunchKernelGGL(fn, dim3((unsigned)n_blocks), dim3(p.threads), 0, stream, single ? *single : DedispJob{},
                       d_jobs, n_jobs, p.tpd, p.dpb);
    AMBER_HIP(hipGetLastError(), "dedisperse (direct reads) launch");
    return AMBER_OK;
}

}  // namespace amber
