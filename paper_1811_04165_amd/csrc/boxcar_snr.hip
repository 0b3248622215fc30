// Boxcar integration and S/N on gfx950.
//
// A dedispersed row is processed in LDS chunks.  Each chunk holds the
// exclusive prefix sum Q of `chunk` consecutive samples (uint32, modulo 2^32);
// a boxcar of width w starting at local index u is then Q[u + w] - Q[u],
// exact in int32 because the true sum fits (wrap-around cancels).  Chunks
// overlap by H >= max width samples so every output of a chunk finds its whole
// window inside it; all widths are served from the same prefix array.
//
// The prefix array lives in LDS unpadded.  Lane l of the prefix pass owns
// samples 16 l - 1 .. 16 l + 14 of the chunk (the first lane's first is
// zero), so its 16 prefix values are Q[16 l .. 16 l + 15], four aligned
// 16-byte stores.  The statistics read Q[u .. u + 3] and Q[u + w .. u + w + 3]
// (u a multiple of 4) as one aligned 16-byte load each when 4 divides w, and
// as dword loads at immediate offsets otherwise, so no per-element index
// arithmetic remains.  (A layout padded by 4 dwords per 64, or assembling
// widths 1 to 3 in registers from two aligned groups, measured slower.)
//
// S/N statistics per (width, row): per work-item the running maximum with its
// first index (strictly greater replaces it, and each work-item visits its
// outputs in increasing t), and FP64 sums of (x - r) and (x - r)^2 about an
// integer reference r close to the series mean.  For the reduction across
// wavefronts the maximum is packed as one int64 key (value << 32 | ~t) so
// that a plain max keeps the earliest peak; the finish is FP64.  Bounds are
// tested per element only in a work-item's last, partial step.
#include "internal.h"

#include <cfloat>
#include <climits>

namespace amber {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));


// Widths of the sliding boxcars, or (dec != 0) decimation factors: then entry
// k is the series of sums of w[k] consecutive samples starting at multiples
// of w[k], i.e. the width-w[k] boxcar read at t = j w[k], j < n_out / w[k].
struct WidthSet {
    int32_t w[AMBER_MAX_WIDTHS];
    int32_t step[AMBER_MAX_WIDTHS];
    int32_t n;
    int32_t dec;
};

struct Stat {
    long long key;
    double s1, s2;
};

__device__ __forceinline__ long long pack_key(int32_t x, int64_t t)
{
    // high half: the signed value; low half: ~t, so equal values prefer the earlier t
    return (long long)(((uint64_t)(int64_t)x << 32) | (uint64_t)(0xffffffffu - (uint32_t)t));
}

__device__ __forceinline__ void stat_init(Stat &s)
{
    s.key = LLONG_MIN;
    s.s1 = 0.0;
    s.s2 = 0.0;
}

__device__ __forceinline__ void stat_add(Stat &s, int32_t x, int64_t t, double r)
{
    const long long k = pack_key(x, t);
    s.key = k > s.key ? k : s.key;
    const double d = (double)x - r;
    s.s1 += d;
    s.s2 = fma(d, d, s.s2);
}

// Running statistics of one work-item: values arrive in increasing t, so a
// strictly greater value is the only one that replaces the maximum.  Values
// are > INT32_MIN (|box| < 2^31 by the callers' contract).
struct Run {
    int32_t vmax;
    uint32_t tmax;
    double s1, s2;
};

__device__ __forceinline__ void run_init(Run &s)
{
    s.vmax = INT32_MIN;
    s.tmax = 0xffffffffu;
    s.s1 = 0.0;
    s.s2 = 0.0;
}

__device__ __forceinline__ void run_add(Run &s, int32_t x, uint32_t t, double r)
{
    const bool up = x > s.vmax;
    s.vmax = up ? x : s.vmax;
    s.tmax = up ? t : s.tmax;
    const double d = (double)x - r;
    s.s1 += d;
    s.s2 = fma(d, d, s.s2);
}

__device__ __forceinline__ Stat run_stat(const Run &s)
{
    Stat o;
    o.key = pack_key(s.vmax, s.tmax);  // the initial state packs to LLONG_MIN
    o.s1 = s.s1;
    o.s2 = s.s2;
    return o;
}

__device__ __forceinline__ Stat wave_reduce(Stat s)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long long k = __shfl_xor(s.key, off, 64);
        s.key = k > s.key ? k : s.key;
        s.s1 += __shfl_xor(s.s1, off, 64);
        s.s2 += __shfl_xor(s.s2, off, 64);
    }
    return s;
}

// Writes (snr, peak) of one series of N values from its reduced statistics.
__device__ __forceinline__ void finish(const Stat &s, int64_t n, double r, float *snr, int32_t *peak)
{
    const int32_t vmax = (int32_t)(s.key >> 32);
    const uint32_t t = 0xffffffffu - (uint32_t)(s.key & 0xffffffffll);
    const double m1 = s.s1 / (double)n;
    double var = s.s2 / (double)n - m1 * m1;
    var = var > 0.0 ? var : 0.0;
    const double sigma = sqrt(var);
    const double excess = ((double)vmax - r) - m1;
    *snr = sigma > 0.0 ? (float)(excess / sigma) : 0.0f;
    if (peak) *peak = (int32_t)t;
}

// Block reduction of per-thread stats for NW widths; thread k < n_w receives
// width k's total.  scratch holds NW * 16 Stats.
template <int NW>
__device__ __forceinline__ void block_reduce(Stat (&st)[NW], int n_w, Stat *scratch)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, waves = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        if (k < n_w) {
            Stat r = wave_reduce(st[k]);
            if (lane == 0) scratch[k * 16 + wave] = r;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < n_w) {
        const int k = threadIdx.x;
        Stat tot = scratch[k * 16];
        for (int w = 1; w < waves; ++w) {
            const Stat o = scratch[k * 16 + w];
            tot.key = o.key > tot.key ? o.key : tot.key;
            tot.s1 += o.s1;
            tot.s2 += o.s2;
        }
        scratch[k * 16] = tot;
    }
    __syncthreads();
}

// Loads samples [cs, cs + chunk) of one row (zero past n_out) and writes the
// exclusive prefix Q[0 .. chunk) to LDS.  Work-item l loads samples
// 16 l .. 16 l + 15 and takes sample 16 l - 1 from its left neighbour (zero
// for the first), so that its 16 prefix values are Q[16 l .. 16 l + 15].
__device__ __forceinline__ void load_prefix(const int32_t *__restrict__ row, int64_t cs, int64_t n_out, bool vec_ok,
                                            uint32_t *Q, uint32_t *wave_tot)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, waves = blockDim.x >> 6;
    const int64_t base = cs + (int64_t)tid * 16;
    uint32_t x[16];
    if (vec_ok && base + 16 <= n_out) {
        const int4 *p = reinterpret_cast<const int4 *>(row + base);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int4 v = p[q];
            x[4 * q + 0] = (uint32_t)v.x; x[4 * q + 1] = (uint32_t)v.y;
            x[4 * q + 2] = (uint32_t)v.z; x[4 * q + 3] = (uint32_t)v.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = (base + e < n_out) ? (uint32_t)row[base + e] : 0u;
    }
    // sample 16 l - 1: the left lane's last; a wave's first lane reads it
    uint32_t left = __shfl_up(x[15], 1, 64);
    if (lane == 0) left = (tid > 0 && base - 1 < n_out) ? (uint32_t)row[base - 1] : 0u;
    uint32_t v[16];
    v[0] = left;
#pragma unroll
    for (int e = 1; e < 16; ++e) v[e] = v[e - 1] + x[e - 1];
    // inclusive scan of work-item totals (samples 16 l - 1 .. 16 l + 14) within the wave
    uint32_t incl = v[15];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int w = 0; w < waves; ++w) {
            const uint32_t y = wave_tot[w];
            wave_tot[w] = run;
            run += y;
        }
    }
    __syncthreads();
    const uint32_t excl = incl - v[15] + wave_tot[wave];
    u32x4 *dst = reinterpret_cast<u32x4 *>(Q + tid * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        dst[q] = u32x4{v[4 * q] + excl, v[4 * q + 1] + excl, v[4 * q + 2] + excl, v[4 * q + 3] + excl};
    __syncthreads();
}

// Loads Q[base .. base + S) (logical indices).  S >= 4 and base a multiple
// of 4: one aligned 16-byte load per group of four; otherwise dword loads.
template <int S>
__device__ __forceinline__ void load_q(const uint32_t *Q, int base, bool aligned, uint32_t (&v)[S])
{
    if (S >= 4 && aligned) {
#pragma unroll
        for (int q = 0; q < S / 4; ++q) {
            const u32x4 x = *reinterpret_cast<const u32x4 *>(Q + base + 4 * q);
            v[4 * q + 0] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s) v[s] = Q[base + s];
    }
}

// Accumulates width w over the chunk's outputs [cs, cs + outs) with S
// consecutive outputs per work-item per step.
template <int S>
__device__ __forceinline__ void width_stats(const uint32_t *Q, int w, int outs, int64_t cs, int64_t n_valid, double r,
                                            Run &st)
{
    const bool w_aligned = (w & 3) == 0;
    for (int g = threadIdx.x; g * S < outs; g += blockDim.x) {
        const int u = g * S;
        uint32_t a[S], b[S];
        load_q<S>(Q, u, true, a);
        load_q<S>(Q, u + w, w_aligned, b);
        const uint32_t t0 = (uint32_t)(cs + u);
        if (u + S <= outs && cs + u + S <= n_valid) {
#pragma unroll
            for (int s = 0; s < S; ++s) run_add(st, (int32_t)(b[s] - a[s]), t0 + s, r);
        } else {  // the last, partial step
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (u + s < outs && cs + u + s < n_valid) run_add(st, (int32_t)(b[s] - a[s]), t0 + s, r);
        }
    }
}

// Accumulates the decimated series of factor f over the bins j whose first
// sample j f lies in [cs, cs + outs), j < n_bins, S bins per work-item per step.
template <int S>
__device__ __forceinline__ void dec_stats(const uint32_t *Q, int f, int outs, int64_t cs, int64_t n_bins, double r,
                                          Run &st)
{
    const int64_t j_lo = (cs + f - 1) / f;
    int64_t j_end = (cs + outs + f - 1) / f;
    j_end = j_end < n_bins ? j_end : n_bins;
    for (int64_t jj = (int64_t)threadIdx.x * S; j_lo + jj < j_end; jj += (int64_t)blockDim.x * S) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t j = j_lo + jj + s;
            if (j < j_end) {
                const int u = (int)(j * f - cs);
                run_add(st, (int32_t)(Q[u + f] - Q[u]), (uint32_t)j, r);
            }
        }
    }
}

__device__ __forceinline__ void dec_stats_any(int step, const uint32_t *Q, int f, int outs, int64_t cs,
                                              int64_t n_bins, double r, Run &st)
{
    switch (step) {
    case 1: dec_stats<1>(Q, f, outs, cs, n_bins, r, st); break;
    case 2: dec_stats<2>(Q, f, outs, cs, n_bins, r, st); break;
    case 4: dec_stats<4>(Q, f, outs, cs, n_bins, r, st); break;
    default: dec_stats<8>(Q, f, outs, cs, n_bins, r, st); break;
    }
}

__device__ __forceinline__ void width_stats_any(int step, const uint32_t *Q, int w, int outs, int64_t cs,
                                                int64_t n_valid, double r, Run &st)
{
    switch (step) {
    case 1: width_stats<1>(Q, w, outs, cs, n_valid, r, st); break;
    case 2: width_stats<2>(Q, w, outs, cs, n_valid, r, st); break;
    case 4: width_stats<4>(Q, w, outs, cs, n_valid, r, st); break;
    default: width_stats<8>(Q, w, outs, cs, n_valid, r, st); break;
    }
}

// ---- fused boxcar + S/N: one work-group per dedispersed row ----------------
// One beam per launch, or a table of beams whose rows are laid out back to
// back in the grid.
// MAXT: the work-group size bound the kernel is compiled for; smaller bounds
// leave more registers per work-item for the NW running statistics.
template <int NW, int MAXT>
__global__ __launch_bounds__(MAXT) void integrate_snr_kernel(BoxJob single, const BoxJob *__restrict__ jobs, int n_jobs,
                                                             WidthSet ws, int chunk, int halo)
{
    extern __shared__ uint4 lds4[];
    uint32_t *Q = reinterpret_cast<uint32_t *>(lds4);
    Stat *scratch = reinterpret_cast<Stat *>(lds4);  // reused after the last chunk
    __shared__ uint32_t wave_tot[16];
    int i = blockIdx.x;
    BoxJob job = single;
    if (jobs) {
        int j = 0;
        while (j + 1 < n_jobs && jobs[j + 1].row_start <= i) ++j;
        job = jobs[j];
        i -= job.row_start;
    }
    const int64_t n_out = job.n_out;
    const int32_t *__restrict__ row = job.dd + (size_t)i * job.dd_stride;
    const int outs = chunk - halo;
    const double d0 = (double)row[0];

    Run st[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) run_init(st[k]);

    for (int64_t cs = 0; cs < n_out; cs += outs) {
        load_prefix(row, cs, n_out, job.vec_ok != 0, Q, wave_tot);
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            if (k < ws.n) {
                const int w = ws.w[k];
                if (ws.dec)
                    dec_stats_any(ws.step[k], Q, w, outs, cs, n_out / w, d0 * w, st[k]);
                else
                    width_stats_any(ws.step[k], Q, w, outs, cs, n_out - w + 1, d0 * w, st[k]);
            }
        }
        __syncthreads();
    }
    Stat sr[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) sr[k] = run_stat(st[k]);
    block_reduce<NW>(sr, ws.n, scratch);
    if ((int)threadIdx.x < ws.n) {
        const int k = threadIdx.x;
        const int w = ws.w[k];
        finish(scratch[k * 16], ws.dec ? n_out / w : n_out - w + 1, d0 * w, job.snr + (size_t)k * job.n_dm + i,
               job.peak ? job.peak + (size_t)k * job.n_dm + i : nullptr);
    }
}

// ---- materialised boxcar: one work-group per (chunk, row) ------------------
__global__ __launch_bounds__(1024) void integrate_kernel(const int32_t *__restrict__ dd, int n_dm, int64_t dd_stride,
                                                         int64_t n_out, WidthSet ws, int chunk, int halo, int vec_ok,
                                                         int32_t *__restrict__ box, int64_t box_stride)
{
    extern __shared__ uint4 lds4[];
    uint32_t *Q = reinterpret_cast<uint32_t *>(lds4);
    __shared__ uint32_t wave_tot[16];
    const int i = blockIdx.y;
    const int outs = chunk - halo;
    const int64_t cs = (int64_t)blockIdx.x * outs;
    load_prefix(dd + (size_t)i * dd_stride, cs, n_out, vec_ok != 0, Q, wave_tot);
    for (int k = 0; k < ws.n; ++k) {
        const int w = ws.w[k];
        int32_t *__restrict__ out = box + ((size_t)k * n_dm + i) * box_stride;
        if (ws.dec) {
            // bins j whose first sample j w lies in this chunk's outputs
            const int64_t j_lo = (cs + w - 1) / w, n_bins = n_out / w;
            int64_t j_end = (cs + outs + w - 1) / w;
            j_end = j_end < n_bins ? j_end : n_bins;
            for (int64_t j = j_lo + threadIdx.x; j < j_end; j += blockDim.x) {
                const int u = (int)(j * w - cs);
                out[j] = (int32_t)(Q[u + w] - Q[u]);
            }
        } else {
            const int64_t n_valid = n_out - w + 1;
            for (int u = threadIdx.x; u < outs; u += blockDim.x) {
                const int64_t t = cs + u;
                if (t < n_valid) out[t] = (int32_t)(Q[u + w] - Q[u]);
            }
        }
    }
}

// ---- S/N of materialised boxcar series: one work-group per (row, width) ----
template <int S>
__global__ __launch_bounds__(1024) void snr_kernel(const int32_t *__restrict__ box, int n_dm, int64_t box_stride,
                                                   int64_t n_out, WidthSet ws, float *__restrict__ snr,
                                                   int32_t *__restrict__ peak)
{
    __shared__ Stat scratch[16];
    const int i = blockIdx.x, k = blockIdx.y;
    const int w = ws.w[k];
    const int64_t n = n_out - w + 1;
    const int32_t *__restrict__ row = box + ((size_t)k * n_dm + i) * box_stride;
    const double r = (double)row[0];
    Stat st;
    stat_init(st);
    for (int64_t base = (int64_t)threadIdx.x * S; base < n; base += (int64_t)blockDim.x * S) {
        int32_t v[S];
#pragma unroll
        for (int s = 0; s < S; ++s) v[s] = (base + s < n) ? row[base + s] : 0;
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (base + s < n) stat_add(st, v[s], base + s, r);
    }
    Stat arr[1] = {st};
    block_reduce<1>(arr, 1, scratch);
    if (threadIdx.x == 0)
        finish(scratch[0], n, r, snr + (size_t)k * n_dm + i, peak ? peak + (size_t)k * n_dm + i : nullptr);
}

WidthSet make_widths(const amber_tiles &t, const int32_t *widths, int n, int decimate)
{
    WidthSet ws{};
    ws.dec = decimate ? 1 : 0;
    for (int k = 0; k < n; ++k) {
        ws.w[k] = widths[k];
        ws.step[k] = t.boxcar_step[k];
    }
    ws.n = n;
    return ws;
}

int halo_of(const BoxcarPlan &p) { return (p.maxw + 15) / 16 * 16; }

amber_status check_chunk(const BoxcarPlan &p)
{
    // plan_boxcar guarantees chunk >= 2 * halo; keep the launchers safe on their own
    if (p.chunk < 2 * halo_of(p)) return fail(AMBER_E_CONFIG, "boxcar chunk shorter than twice its halo");
    return AMBER_OK;
}

template <typename F>
amber_status allow_lds(F fn, int64_t bytes, const char *what)
{
    if (bytes > 64 * 1024)
        AMBER_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)bytes),
                  what);
    return AMBER_OK;
}

}  // namespace

BoxJob make_box_job(const int32_t *d_dd, int n_dm, int64_t dd_stride, int64_t n_out, float *d_snr, int32_t *d_peak)
{
    BoxJob j{};
    j.dd = d_dd;
    j.dd_stride = dd_stride;
    j.n_out = n_out;
    j.snr = d_snr;
    j.peak = d_peak;
    j.n_dm = n_dm;
    j.vec_ok = (dd_stride % 4 == 0) && (((uintptr_t)d_dd & 15) == 0);
    j.row_start = 0;
    return j;
}

amber_status launch_integrate_snr_jobs(const BoxcarPlan &p, const amber_tiles &t, const BoxJob *single,
                                       const BoxJob *d_jobs, int n_jobs, int64_t n_rows, const int32_t *widths,
                                       int n_widths, hipStream_t stream, int decimate)
{
    amber_status s = check_chunk(p);
    if (s != AMBER_OK) return s;
    if (n_rows > 0x7fffffff) return fail(AMBER_E_SHAPE, "too many rows (%lld)", (long long)n_rows);
    // One beam with more than 8 series: passes of at most 8 series through
    // the 8-series kernel (each pass re-reads the rows, but the statistics of
    // 16 series per work-item need registers enough to halve the resident
    // work-groups).
    if (single && n_widths > 8) {
        for (int k0 = 0; k0 < n_widths; k0 += 8) {
            BoxJob j = *single;
            j.snr += (size_t)k0 * j.n_dm;
            if (j.peak) j.peak += (size_t)k0 * j.n_dm;
            amber_tiles tk = t;
            const int nk = n_widths - k0 < 8 ? n_widths - k0 : 8;
            for (int k = 0; k < nk; ++k) tk.boxcar_step[k] = t.boxcar_step[k0 + k];
            if ((s = launch_integrate_snr_jobs(p, tk, &j, nullptr, 1, n_rows, widths + k0, nk, stream, decimate)) !=
                AMBER_OK)
                return s;
        }
        return AMBER_OK;
    }
    const WidthSet ws = make_widths(t, widths, n_widths, decimate);
    const int halo = halo_of(p);
    // the stats scratch reuses the prefix buffer after the last chunk
    int64_t lds = p.lds_bytes;
    const int64_t need = (int64_t)AMBER_MAX_WIDTHS * 16 * sizeof(Stat);
    if (lds < need) lds = need;
    const BoxJob one = single ? *single : BoxJob{};
    const dim3 grid((unsigned)n_rows);
    const int maxt = p.threads <= 256 ? 256 : (p.threads <= 512 ? 512 : 1024);
    auto go = [&](auto kernel) -> amber_status {
        amber_status st = allow_lds(kernel, lds, "hipFuncSetAttribute(integrate_snr)");
        if (st != AMBER_OK) return st;
        hipLaunchKernelGGL(kernel, grid, dim3(p.threads), (size_t)lds, stream, one, d_jobs, n_jobs, ws, p.chunk, halo);
        return AMBER_OK;
    };
    if (n_widths <= 4)
        s = maxt == 256 ? go(integrate_snr_kernel<4, 256>)
                        : (maxt == 512 ? go(integrate_snr_kernel<4, 512>) : go(integrate_snr_kernel<4, 1024>));
    else if (n_widths <= 8)
        s = maxt == 256 ? go(integrate_snr_kernel<8, 256>)
                        : (maxt == 512 ? go(integrate_snr_kernel<8, 512>) : go(integrate_snr_kernel<8, 1024>));
    else
        s = maxt == 256 ? go(integrate_snr_kernel<16, 256>)
                        : (maxt == 512 ? go(integrate_snr_kernel<16, 512>) : go(integrate_snr_kernel<16, 1024>));
    if (s != AMBER_OK) return s;
    AMBER_HIP(hipGetLastError(), "integrate_snr launch");
    return AMBER_OK;
}

amber_status launch_integrate_snr(const BoxcarPlan &p, const amber_tiles &t, const int32_t *d_dd, int n_dm,
                                  int64_t dd_stride, int64_t n_out, const int32_t *widths, int n_widths,
                                  float *d_snr, int32_t *d_peak, hipStream_t stream, int decimate)
{
    const BoxJob j = make_box_job(d_dd, n_dm, dd_stride, n_out, d_snr, d_peak);
    return launch_integrate_snr_jobs(p, t, &j, nullptr, 1, n_dm, widths, n_widths, stream, decimate);
}

amber_status launch_integrate(const BoxcarPlan &p, const amber_tiles &t, const int32_t *d_dd, int n_dm,
                              int64_t dd_stride, int64_t n_out, const int32_t *widths, int n_widths, int32_t *d_box,
                              int64_t box_stride, hipStream_t stream, int decimate)
{
    amber_status s = check_chunk(p);
    if (s != AMBER_OK) return s;
    const WidthSet ws = make_widths(t, widths, n_widths, decimate);
    const int halo = halo_of(p);
    const int outs = p.chunk - halo;
    const int64_t n_chunks = (n_out + outs - 1) / outs;
    const int vec_ok = (dd_stride % 4 == 0) && (((uintptr_t)d_dd & 15) == 0);
    if ((s = allow_lds(integrate_kernel, p.lds_bytes, "hipFuncSetAttribute(integrate)")) != AMBER_OK) return s;
    hipLaunchKernelGGL(integrate_kernel, dim3((unsigned)n_chunks, n_dm), dim3(p.threads), (size_t)p.lds_bytes, stream,
                       d_dd, n_dm, dd_stride, n_out, ws, p.chunk, halo, vec_ok, d_box, box_stride);
    AMBER_HIP(hipGetLastError(), "integrate launch");
    return AMBER_OK;
}

amber_status launch_snr(const BoxcarPlan &p, const amber_tiles &t, const int32_t *d_box, int n_dm, int64_t box_stride,
                        int64_t n_out, const int32_t *widths, int n_widths, float *d_snr, int32_t *d_peak,
                        hipStream_t stream)
{
    const WidthSet ws = make_widths(t, widths, n_widths, 0);
    // the per-row kernel uses the first width's step as its items per thread
    const int step = t.boxcar_step[0];
    dim3 grid(n_dm, n_widths);
    switch (step) {
    case 1: hipLaunchKernelGGL(snr_kernel<1>, grid, dim3(p.threads), 0, stream, d_box, n_dm, box_stride, n_out, ws, d_snr, d_peak); break;
    case 2: hipLaunchKernelGGL(snr_kernel<2>, grid, dim3(p.threads), 0, stream, d_box, n_dm, box_stride, n_out, ws, d_snr, d_peak); break;
    case 4: hipLaunchKernelGGL(snr_kernel<4>, grid, dim3(p.threads), 0, stream, d_box, n_dm, box_stride, n_out, ws, d_snr, d_peak); break;
    default: hipLaunchKernelGGL(snr_kernel<8>, grid, dim3(p.threads), 0, stream, d_box, n_dm, box_stride, n_out, ws, d_snr, d_peak); break;
    }
    AMBER_HIP(hipGetLastError(), "snr launch");
    return AMBER_OK;
}

}  // namespace amber
