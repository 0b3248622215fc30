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
#include <type_traits>

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

// ---- fused boxcar + S/N over wavefront spans (sliding widths <= 64) --------
//
// One work-group per dedispersed row and W = blockDim / 64 wavefronts.  The
// row's outputs are cut into blocks of 256 (64 lanes x 4); wavefront v sweeps
// the blocks [v nb / W, (v + 1) nb / W) in order, on its own (no barrier
// until the end).  Per step j:
//  - block j + 1's samples (loaded SPAN_NB - 1 steps earlier, 16 B per lane,
//    coalesced) are centred on c = dd[row][0], prefix-summed across the
//    wavefront with DPP and written to a two-block LDS ring (slot (j + 1) & 1);
//    the first entries of slot 0 are repeated after slot 1, so that no read
//    wraps;
//  - lane l reads the prefix at its 4 outputs u = 256 j + 4 l .. + 3 and, per
//    width w, at u + w: box' = Q[u + w] - Q[u] is the width-w boxcar minus
//    w c, exact in uint32 arithmetic because its true value fits int32;
//  - per width it keeps the running maximum (3-input maxima of its 4 values),
//    the block where that maximum last rose, and the sum of squares in int64
//    (one 32 x 32 + 64-bit multiply-add per value).
// The int64 sums are exact while (max width x max |centred sample|)^2 times
// the values per lane stays below 2^62, and the wavefront's block totals
// (which give the row's sum) while max |centred sample| < 2^23; each
// wavefront tracks its largest centred sample, and a row that breaks either
// bound has its sum and sums of squares recomputed after the sweep (no
// dedispersed uint8 data of fewer than 32 896 channels comes near it).  The sum of box' over the row needs no per-output work: it is w T
// minus head and tail terms, with T the centred row's sum.  After the sweep:
// wavefront reductions, one barrier, then per width one wavefront finds the
// first index of the maximum (its 4 candidate outputs in the earliest block
// that reaches it, recomputed from dd), forms the mean from the closed form,
// the variance and the S/N.

constexpr int kSpanBlk = 256;
constexpr int kSpanMaxW = 64;
#ifndef SPAN_NB
#define SPAN_NB 4
#endif
// reads of an odd block reach 256 + 4 * 63 + kSpanMaxW + 7 = 579 < 2 * 256 + kSpanDup
constexpr int kSpanDup = 80;
constexpr int kSpanRing = 2 * kSpanBlk + kSpanDup;  // dwords per wavefront

struct SpanRes {
    long long key;
    double s2;
};

// Inclusive prefix sum across the wavefront (rows of 16 lanes with row_shr,
// then row_bcast15 / row_bcast31 between rows).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false); // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false); // row_bcast:31
    return v;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw samples of one lane in one block (block b: samples 256 b + 4 lane ..
// + 3).  VEC (16-byte aligned rows of >= 4 samples): one 16-byte load from an
// in-bounds address; a lane whose 4 samples are not all inside [0, n_out)
// loads the row's first 16 bytes instead and re-reads its samples one by one
// when the block is consumed.  Otherwise four dword loads from clamped
// addresses.  Loads go through global-address-space pointers: flat loads
// would also count against the LDS counter, and the compiler would then
// drain every load in flight at each LDS wait.  Indices are 32-bit: the
// launcher takes rows of fewer than 2^30 samples.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) int32_t g_i32;
typedef const __attribute__((address_space(1))) i32x4 g_i4;

// Buffer loads: a row is a buffer of n_out dwords whose reads past its end
// return zero (the hardware's range check), so no load needs its address
// clamped and the offsets are a fixed per-lane part plus a scalar block part.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const int32_t *row, int n_out)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(row), (short)0, n_out * 4, 0x00020000);
}

template <bool VEC>
__device__ __forceinline__ i32x4 span_load(__amdgpu_buffer_rsrc_t rs, int blk, int lane)
{
    // the whole byte offset in the vector operand, which the range check
    // covers (blk >= 0; rows of fewer than 2^29 samples)
    const int off = blk * (kSpanBlk * 4) + 16 * lane;
    if (VEC) return __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    i32x4 v;
    v.x = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    v.y = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4, 0, 0);
    v.z = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 8, 0, 0);
    v.w = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 12, 0, 0);
    return v;
}

__device__ __forceinline__ int32_t max3i(int32_t a, int32_t b, int32_t c)
{
    int32_t r;
    asm("v_max3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ int32_t min3i(int32_t a, int32_t b, int32_t c)
{
    int32_t r;
    asm("v_min3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Centres block `blk` on c, writes its prefix (starting at `base`) to ring
// slot blk & 1, widens [xlo, xhi] to its centred samples and returns the
// block's total (uint32, true value fits int32).
template <bool VEC>
__device__ __forceinline__ uint32_t span_put(uint32_t *ring, int blk, const i32x4 &r, const int32_t *__restrict__ row,
                                             int n_out, int32_t c, uint32_t base, int lane, int32_t &xlo,
                                             int32_t &xhi)
{
    const int t = blk * kSpanBlk + 4 * lane;
    int32_t x[4];
    if (VEC && (blk + 1) * kSpanBlk <= n_out) {  // the whole block lies in the row
        x[0] = r.x - c; x[1] = r.y - c; x[2] = r.z - c; x[3] = r.w - c;
    } else if (VEC) {
        if (t + 4 <= n_out) {
            x[0] = r.x - c; x[1] = r.y - c; x[2] = r.z - c; x[3] = r.w - c;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = (t + e < n_out) ? ((g_i32 *)row)[t + e] - c : 0;
        }
    } else {
        const int32_t v[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = (t + e < n_out) ? v[e] - c : 0;
    }
    xlo = min3i(min3i(xlo, x[0], x[1]), x[2], x[3]);
    xhi = max3i(max3i(xhi, x[0], x[1]), x[2], x[3]);
    const uint32_t l0 = (uint32_t)x[0], l1 = l0 + (uint32_t)x[1], l2 = l1 + (uint32_t)x[2],
                   l3 = l2 + (uint32_t)x[3];
    const uint32_t incl = wave_scan_incl(l3);
    const uint32_t ex = incl - l3 + base;
    const u32x4 q = u32x4{ex, ex + l0, ex + l1, ex + l2};
    const int slot = blk & 1;
    *reinterpret_cast<u32x4 *>(ring + slot * kSpanBlk + 4 * lane) = q;
    if (slot == 0 && lane < kSpanDup / 4) *reinterpret_cast<u32x4 *>(ring + 2 * kSpanBlk + 4 * lane) = q;
    return (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
}

// box'[e] = Q[b + e + w] - Q[b + e] for the lane's 4 outputs (A = Q[b .. b + 3]).
template <int R>
__device__ __forceinline__ void span_box(const uint32_t *ring, int b, int w, const u32x4 &A, int32_t (&x)[4])
{
    const int q = w - R;
    const u32x4 g0 = *reinterpret_cast<const u32x4 *>(ring + b + q);
    if (R == 0) {
        x[0] = (int32_t)(g0.x - A.x); x[1] = (int32_t)(g0.y - A.y);
        x[2] = (int32_t)(g0.z - A.z); x[3] = (int32_t)(g0.w - A.w);
    } else {
        const u32x4 g1 = *reinterpret_cast<const u32x4 *>(ring + b + q + 4);
        const uint32_t g[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
        x[0] = (int32_t)(g[R] - A.x); x[1] = (int32_t)(g[R + 1] - A.y);
        x[2] = (int32_t)(g[R + 2] - A.z); x[3] = (int32_t)(g[R + 3] - A.w);
    }
}

template <bool POW2>
__device__ __forceinline__ int span_width(const WidthSet &ws, int k)
{
    return POW2 ? (1 << k) : ws.w[k];
}

// One block of one width: the lane's 4 boxcar values x, all valid (TAIL
// false) or valid below n_valid (TAIL true).
template <bool TAIL>
__device__ __forceinline__ void span_acc(const int32_t (&x)[4], int t0, int n_valid, int32_t &vmax, int32_t &jmax,
                                         long long &s2, int32_t j)
{
    int32_t m;
    if (!TAIL) {
        m = max3i(max3i(vmax, x[0], x[1]), x[2], x[3]);
#pragma unroll
        for (int e = 0; e < 4; ++e) s2 += (long long)x[e] * (long long)x[e];
    } else {
        m = vmax;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool ok = t0 + e < n_valid;
            m = ok ? max(m, x[e]) : m;
            const int32_t v = ok ? x[e] : 0;
            s2 += (long long)v * (long long)v;
        }
    }
    jmax = m != vmax ? j : jmax;
    vmax = m;
}

// The statistics of block j for every width (its prefix and the next
// block's are in the ring).
template <int NW, bool POW2, bool TAIL>
__device__ __forceinline__ void span_block(const uint32_t *ring, int j, int lane, const WidthSet &ws, int n_out,
                                           int32_t (&vmax)[NW], int32_t (&jmax)[NW], long long (&s2)[NW])
{
    const int b = (j & 1) * kSpanBlk + 4 * lane;
    const int t0 = j * kSpanBlk + 4 * lane;
    if (POW2) {
        // widths 1, 2, 4, ..: every window end lies in one of the groups of
        // four at offsets 0, 4, 8, 16, ..; all of them are read before any is
        // used, so that a step waits for LDS once (read one by one, each read
        // would wait a full LDS latency)
        constexpr int NG = NW < 3 ? 2 : NW - 1;
        u32x4 G[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) G[g] = *reinterpret_cast<const u32x4 *>(ring + b + (g == 0 ? 0 : 2 << g));
        __builtin_amdgcn_sched_barrier(0);
        const u32x4 A = G[0];
        const uint32_t lo[8] = {G[0].x, G[0].y, G[0].z, G[0].w, G[1].x, G[1].y, G[1].z, G[1].w};
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            int32_t x[4];
            if (k < 2) {  // w = 1, 2: ends inside groups 0 and 1
                const int w = 1 << k;
                x[0] = (int32_t)(lo[w] - A.x); x[1] = (int32_t)(lo[w + 1] - A.y);
                x[2] = (int32_t)(lo[w + 2] - A.z); x[3] = (int32_t)(lo[w + 3] - A.w);
            } else {      // w = 4 << (k - 2): group k - 1
                const u32x4 E = G[k - 1];
                x[0] = (int32_t)(E.x - A.x); x[1] = (int32_t)(E.y - A.y);
                x[2] = (int32_t)(E.z - A.z); x[3] = (int32_t)(E.w - A.w);
            }
            span_acc<TAIL>(x, t0, n_out - (1 << k) + 1, vmax[k], jmax[k], s2[k], j);
        }
        return;
    }
    const u32x4 A = *reinterpret_cast<const u32x4 *>(ring + b);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int w = span_width<POW2>(ws, k);
        int32_t x[4];
        switch (w & 3) {
        case 0: span_box<0>(ring, b, w, A, x); break;
        case 1: span_box<1>(ring, b, w, A, x); break;
        case 2: span_box<2>(ring, b, w, A, x); break;
        default: span_box<3>(ring, b, w, A, x); break;
        }
        span_acc<TAIL>(x, t0, n_out - w + 1, vmax[k], jmax[k], s2[k], j);
    }
}

// Whole-wavefront reductions with DPP (quad permutes, row mirrors, then
// row_bcast15 / row_bcast31 into the last row); the result is read from lane
// 63 and is the same in every lane.  64-bit values move as two halves.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t v, uint64_t identity)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)identity, (int)(uint32_t)v, CTRL, ROWS,
                                                               0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(identity >> 32), (int)(uint32_t)(v >> 32),
                                                               CTRL, ROWS, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t lane63(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ long long wave_max_ll(long long v)
{
    const uint64_t id = (uint64_t)LLONG_MIN;
    auto mx = [](long long a, uint64_t b) { return a > (long long)b ? a : (long long)b; };
    v = mx(v, dpp64<0xb1, 0xf>((uint64_t)v, id));   // quad_perm [1,0,3,2]
    v = mx(v, dpp64<0x4e, 0xf>((uint64_t)v, id));   // quad_perm [2,3,0,1]
    v = mx(v, dpp64<0x141, 0xf>((uint64_t)v, id));  // row_half_mirror
    v = mx(v, dpp64<0x140, 0xf>((uint64_t)v, id));  // row_mirror
    v = mx(v, dpp64<0x142, 0xa>((uint64_t)v, id));  // row_bcast:15
    v = mx(v, dpp64<0x143, 0xc>((uint64_t)v, id));  // row_bcast:31
    return (long long)lane63((uint64_t)v);
}

__device__ __forceinline__ double wave_sum_d(double v)
{
    auto add = [](double a, uint64_t b) { return a + __longlong_as_double((long long)b); };
    auto bits = [](double a) { return (uint64_t)__double_as_longlong(a); };
    v = add(v, dpp64<0xb1, 0xf>(bits(v), 0));
    v = add(v, dpp64<0x4e, 0xf>(bits(v), 0));
    v = add(v, dpp64<0x141, 0xf>(bits(v), 0));
    v = add(v, dpp64<0x140, 0xf>(bits(v), 0));
    v = add(v, dpp64<0x142, 0xa>(bits(v), 0));
    v = add(v, dpp64<0x143, 0xc>(bits(v), 0));
    return __longlong_as_double((long long)lane63(bits(v)));
}

__device__ __forceinline__ long long wave_sum_ll(long long v)
{
    v += (long long)dpp64<0xb1, 0xf>((uint64_t)v, 0);
    v += (long long)dpp64<0x4e, 0xf>((uint64_t)v, 0);
    v += (long long)dpp64<0x141, 0xf>((uint64_t)v, 0);
    v += (long long)dpp64<0x140, 0xf>((uint64_t)v, 0);
    v += (long long)dpp64<0x142, 0xa>((uint64_t)v, 0);
    v += (long long)dpp64<0x143, 0xc>((uint64_t)v, 0);
    return (long long)lane63((uint64_t)v);
}

// NW: the exact number of widths; POW2: widths are 1, 2, 4, ... 2^(NW-1).
constexpr int NB = SPAN_NB;
template <int NW, bool POW2, bool VEC>
__global__ __launch_bounds__(1024) void span_snr_kernel(BoxJob single, const BoxJob *__restrict__ jobs, int n_jobs,
                                                        WidthSet ws)
{
    extern __shared__ uint4 lds4[];
    // the wavefront index is uniform: keep it (and the span bounds, the block
    // counter and every branch on them) in scalar registers
    const int W = blockDim.x >> 6, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    uint32_t *ring = reinterpret_cast<uint32_t *>(lds4) + wave * kSpanRing;
    SpanRes *res = reinterpret_cast<SpanRes *>(reinterpret_cast<uint32_t *>(lds4) + W * kSpanRing);
    long long *tres = reinterpret_cast<long long *>(res + W * NW);
    int *flags = reinterpret_cast<int *>(tres + W);  // per wavefront: its sums of squares may have overflowed

    int i = blockIdx.x;
    BoxJob job = single;
    if (jobs) {
        int j = 0;
        while (j + 1 < n_jobs && jobs[j + 1].row_start <= i) ++j;
        job = jobs[j];
        i -= job.row_start;
    }
    const int n_out = (int)job.n_out;
    const int32_t *__restrict__ row = job.dd + (size_t)i * job.dd_stride;
    const int32_t c = *(g_i32 *)row;
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(row, n_out);
    // the row's first and last 64 samples (for the boxcar sums' head and tail
    // terms), loaded now and used after the sweep
    const int32_t head = lane < n_out ? ((g_i32 *)row)[lane] : 0;
    const int32_t tail = n_out - 1 - lane >= 0 ? ((g_i32 *)row)[n_out - 1 - lane] : 0;
    int maxw = 1;
#pragma unroll
    for (int k = 0; k < NW; ++k) maxw = max(maxw, span_width<POW2>(ws, k));
    const int n_min = n_out - maxw + 1;  // outputs below it are valid for every width

    int32_t vmax[NW], jmax[NW];
    long long s2[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        vmax[k] = INT32_MIN;
        jmax[k] = -1;
        s2[k] = 0;
    }
    long long tsum = 0;
    int32_t xlo = 0, xhi = 0;
    bool overflow = false;

    const int nb = (n_out + kSpanBlk - 1) / kSpanBlk;
    const int jb = (int)((uint32_t)nb * (uint32_t)wave / (uint32_t)W),
              je = (int)((uint32_t)nb * (uint32_t)(wave + 1) / (uint32_t)W);
    if (jb < je) {
        // blocks before j_tail have every output valid for every width; the
        // others (at most two, at the row's end) take the masked statistics
        const int j_tail = min(max(n_min / kSpanBlk, jb), je);
        uint32_t base = 0;
        // Main part, blocks [jb, j_tail): NB block buffers.  While block j
        // is summed, blocks j + 1 (its windows' lookahead, put into the ring
        // first) .. j + NB - 1 are loaded and j + NB is being loaded.  The
        // loop is unrolled NB times so that buffers are never copied (a copy
        // would wait for the load in flight); it starts NB - 1 steps early at
        // most (dummy steps: loads and prefix writes of earlier blocks, no
        // statistics), so that its length is a multiple of NB.
        if (jb < j_tail) {
            const int r = (NB - (j_tail - jb) % NB) % NB;
            int j = jb - r;
            i32x4 buf[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) buf[u] = span_load<VEC>(rs, max(j + u, 0), lane);
            base = span_put<VEC>(ring, j, buf[0], row, n_out, c, 0u, lane, xlo, xhi);
            if (j >= jb) tsum += (int32_t)base;
            for (; j < j_tail; j += NB) {
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int jj = j + u;
                    // blocks past the lookahead are loaded and never used
                    // (past the row's end the loads return zeros)
                    buf[u] = span_load<VEC>(rs, max(jj + NB, 0), lane);
                    const uint32_t tot =
                        span_put<VEC>(ring, jj + 1, buf[(u + 1) % NB], row, n_out, c, base, lane, xlo, xhi);
                    base += tot;
                    if (jj + 1 >= jb && jj + 1 < je) tsum += (int32_t)tot;
                    wave_sync_lds();
                    if (jj >= jb) span_block<NW, POW2, false>(ring, jj, lane, ws, n_out, vmax, jmax, s2);
                    wave_sync_lds();
                }
            }
        } else {
            base = span_put<VEC>(ring, jb, span_load<VEC>(rs, jb, lane), row, n_out, c, 0u, lane, xlo,
                                 xhi);
            tsum += (int32_t)base;
        }
        // tail blocks: block j + 1 loaded and put, then block j's masked statistics
        for (int j = j_tail; j < je; ++j) {
            const uint32_t tot = span_put<VEC>(ring, j + 1, span_load<VEC>(rs, j + 1, lane), row, n_out, c,
                                               base, lane, xlo, xhi);
            base += tot;
            if (j + 1 < je) tsum += (int32_t)tot;
            wave_sync_lds();
            span_block<NW, POW2, true>(ring, j, lane, ws, n_out, vmax, jmax, s2);
            wave_sync_lds();
        }
        // exactness: a block's total (256 centred samples) fits int32 while
        // max |x'| < 2^23; the int64 sums of squares while (maxw max |x'|)^2
        // times the 4 (je - jb) values per lane and width stays below 2^62
        const int32_t xm = (int32_t)wave_max_ll((long long)max(max(xhi, -xlo), 0));
        const double bound = (double)maxw * (double)xm;
        overflow = xm >= (1 << 23) || bound * bound * (4.0 * (double)(je - jb)) >= 4.6e18;
    }

    // wavefront totals: per width (max, earliest 4-output group) and sum of squares
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int u0 = jmax[k] >= 0 ? jmax[k] * kSpanBlk + 4 * lane : 0;
        const long long key = wave_max_ll(pack_key(vmax[k], u0));
        const double s = wave_sum_d((double)s2[k]);
        if (lane == 0) res[wave * NW + k] = SpanRes{key, s};
    }
    if (lane == 0) {
        tres[wave] = tsum;
        flags[wave] = overflow ? 1 : 0;
    }
    __syncthreads();
    bool redo = false;
    long long T = 0;
    for (int v = 0; v < W; ++v) {
        redo = redo || flags[v] != 0;
        T += tres[v];
    }
    if (redo) {
        // the centred row's sum again, in int64
        long long a = 0;
        for (int t = lane; t < n_out; t += 64) a += (long long)row[t] - c;
        T = wave_sum_ll(a);
    }
    // this wavefront's widths k = wave, wave + W, ..: totals over the
    // wavefronts (in a fixed order), then the loads that find the first index
    // of each maximum, all issued before any is used
    long long key[NW];
    double s2t[NW];
    int32_t v1[NW], v2[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        if (k % W != wave) continue;
        key[k] = LLONG_MIN;
        s2t[k] = 0.0;
        for (int v = 0; v < W; ++v) {
            const SpanRes r = res[v * NW + k];
            key[k] = r.key > key[k] ? r.key : key[k];
            s2t[k] += r.s2;
        }
        const int u0 = (int)(0xffffffffu - (uint32_t)(key[k] & 0xffffffffll));
        v1[k] = (u0 + lane < n_out) ? row[u0 + lane] : 0;
        v2[k] = (lane < 3 && u0 + 64 + lane < n_out) ? row[u0 + 64 + lane] : 0;
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        if (k % W != wave) continue;
        const int w = span_width<POW2>(ws, k);
        const int N = n_out - w + 1;
        double s = s2t[k];
        if (redo) {
            // sums of squares again in FP64: lane l takes a contiguous run
            // of outputs and slides its window along it
            const int C = (N + 63) / 64, t0 = lane * C, t1 = min(N, t0 + C);
            double acc = 0.0;
            if (t0 < t1) {
                long long bx = 0;
                for (int m = 0; m < w; ++m) bx += (long long)row[t0 + m] - c;
                acc = (double)bx * (double)bx;
                for (int t = t0 + 1; t < t1; ++t) {
                    bx += (long long)row[t + w - 1] - (long long)row[t - 1];
                    acc += (double)bx * (double)bx;
                }
            }
            s = wave_sum_d(acc);
        }
        const int32_t vm = (int32_t)(key[k] >> 32);
        const int u0 = (int)(0xffffffffu - (uint32_t)(key[k] & 0xffffffffll));
        // head and tail outputs of the boxcar sum's weights below w
        double corr = 0.0;
        if (lane <= w - 2) {
            const int th = lane, tt = n_out - 1 - lane;
            if (th < n_out) {
                const int cnt = min(th, N - 1) - max(0, th - w + 1) + 1;
                corr += (double)(w - cnt) * (double)(head - c);
            }
            if (tt >= w - 1) {
                const int cnt = min(tt, N - 1) - max(0, tt - w + 1) + 1;
                corr += (double)(w - cnt) * (double)(tail - c);
            }
        }
        corr = wave_sum_d(corr);
        const double s1 = (double)w * (double)T - corr;
        // first index of the maximum among outputs u0 .. u0 + 3
        const uint32_t p1 = wave_scan_incl((uint32_t)v1[k]), p2 = wave_scan_incl((uint32_t)v2[k]);
        const uint32_t p64 = (uint32_t)__builtin_amdgcn_readlane((int)p1, 63);
        auto S = [&](int m) -> uint32_t {
            if (m == 0) return 0u;
            if (m <= 64) return (uint32_t)__builtin_amdgcn_readlane((int)p1, m - 1);
            return p64 + (uint32_t)__builtin_amdgcn_readlane((int)p2, m - 65);
        };
        const uint32_t want = (uint32_t)vm + (uint32_t)w * (uint32_t)c;
        int tstar = u0;
        for (int e = 3; e >= 0; --e)
            if (u0 + e < N && S(e + w) - S(e) == want) tstar = u0 + e;
        if (lane == 0) {
            const double m1 = s1 / (double)N;
            double var = s / (double)N - m1 * m1;
            var = var > 0.0 ? var : 0.0;
            const double sigma = sqrt(var);
            job.snr[(size_t)k * job.n_dm + i] = sigma > 0.0 ? (float)(((double)vm - m1) / sigma) : 0.0f;
            if (job.peak) job.peak[(size_t)k * job.n_dm + i] = tstar;
        }
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
    // 16-byte row loads: aligned rows, and at least 4 samples (the span kernel
    // reads a row's first 16 bytes in place of a load past its end)
    j.vec_ok = (dd_stride % 4 == 0) && (((uintptr_t)d_dd & 15) == 0) && n_out >= 4;
    j.row_start = 0;
    return j;
}

namespace {

// The span kernel: sliding widths up to kSpanMaxW, at most 8 per launch.
template <int NW>
void launch_span_nw(bool pow2, bool vec, dim3 grid, dim3 block, size_t lds, hipStream_t stream, const BoxJob &one,
                    const BoxJob *d_jobs, int n_jobs, const WidthSet &ws)
{
    if (pow2) {
        if (vec) hipLaunchKernelGGL((span_snr_kernel<NW, true, true>), grid, block, lds, stream, one, d_jobs, n_jobs, ws);
        else hipLaunchKernelGGL((span_snr_kernel<NW, true, false>), grid, block, lds, stream, one, d_jobs, n_jobs, ws);
    } else {
        if (vec) hipLaunchKernelGGL((span_snr_kernel<NW, false, true>), grid, block, lds, stream, one, d_jobs, n_jobs, ws);
        else hipLaunchKernelGGL((span_snr_kernel<NW, false, false>), grid, block, lds, stream, one, d_jobs, n_jobs, ws);
    }
}

amber_status launch_span_snr(const BoxcarPlan &p, const BoxJob *single, const BoxJob *d_jobs, int n_jobs,
                             int64_t n_rows, const int32_t *widths, int n_widths, bool vec, hipStream_t stream)
{
    WidthSet ws{};
    bool pow2 = true;
    for (int k = 0; k < n_widths; ++k) {
        ws.w[k] = widths[k];
        pow2 = pow2 && widths[k] == (1 << k);
    }
    ws.n = n_widths;
    const int W = p.threads / kWave;
    const size_t lds = (size_t)W * kSpanRing * 4 + (size_t)W * n_widths * sizeof(SpanRes) +
                       (size_t)W * sizeof(long long) + (size_t)W * sizeof(int);
    const BoxJob one = single ? *single : BoxJob{};
    const dim3 grid((unsigned)n_rows), block(p.threads);
    switch (n_widths) {
    case 1: launch_span_nw<1>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    case 2: launch_span_nw<2>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    case 3: launch_span_nw<3>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    case 4: launch_span_nw<4>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    case 5: launch_span_nw<5>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    case 6: launch_span_nw<6>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    case 7: launch_span_nw<7>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    case 8: launch_span_nw<8>(pow2, vec, grid, block, lds, stream, one, d_jobs, n_jobs, ws); break;
    default: return fail(AMBER_E_CONFIG, "span kernel takes 1 to 8 widths, got %d", n_widths);
    }
    AMBER_HIP(hipGetLastError(), "integrate_snr (span) launch");
    return AMBER_OK;
}

}  // namespace

bool span_snr_applies(const int32_t *widths, int n_widths, int decimate, int64_t max_n_out)
{
    if (decimate || n_widths < 1 || n_widths > 8 || max_n_out >= ((int64_t)1 << 29)) return false;
    for (int k = 0; k < n_widths; ++k)
        if (widths[k] > kSpanMaxW) return false;
    return true;
}

amber_status launch_integrate_snr_jobs(const BoxcarPlan &p, const amber_tiles &t, const BoxJob *single,
                                       const BoxJob *d_jobs, int n_jobs, int64_t n_rows, const int32_t *widths,
                                       int n_widths, hipStream_t stream, int decimate, int all_vec,
                                       int64_t max_n_out)
{
    amber_status s = check_chunk(p);
    if (s != AMBER_OK) return s;
    if (n_rows > 0x7fffffff) return fail(AMBER_E_SHAPE, "too many rows (%lld)", (long long)n_rows);
    if (span_snr_applies(widths, n_widths, decimate, single ? single->n_out : max_n_out)) {
        const bool vec = single ? single->vec_ok != 0 : all_vec > 0;
        return launch_span_snr(p, single, d_jobs, n_jobs, n_rows, widths, n_widths, vec, stream);
    }
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
            if ((s = launch_integrate_snr_jobs(p, tk, &j, nullptr, 1, n_rows, widths + k0, nk, stream, decimate, -1, j.n_out)) !=
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
