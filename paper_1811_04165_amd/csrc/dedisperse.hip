// Brute-force dedispersion on gfx950.
//
//   dd[i][t] = sum over c of in[c][t + delay[i][c]]
//
// Work decomposition.  A work-group owns `dpb` consecutive DM trials and
// `tpd * spt` consecutive output samples; each wavefront owns one DM trial
// and 64 * spt samples.  The group walks the channels `cu` at a time.
//
// Staging.  For each of the `cu` channels the group copies into LDS the input
// window every DM of the tile needs: it starts at the first DM's delay (later
// DMs read at most (dpb - 1) * max_step samples further in).  Samples are
// widened from uint8 to 16 bits and stored twice, the second copy shifted by
// one sample, so the two samples at any offset are one aligned dword of one of
// the copies.  A work-item stages two 8-sample chunks half a row apart, so
// that each write instruction covers consecutive 16-byte lines across the
// lanes (all LDS banks).  The global loads of the next channel group (input
// and delays, as range-checked buffer loads with 32-bit offsets) are issued
// before the current group is summed, so their latency hides behind the sums.
//
// Accumulation.  Sums of up to 256 channels fit 16 bits, so each dword holds
// two running sums and one 32-bit add advances both.  The wave's outputs are
// cut into blocks of 128 dwords (256 samples); lane l owns dwords 2l and
// 2l + 1 of each block and reads both with one 8-byte `ds_read_b64`: the LDS
// serves about 32 lane-addresses per clock, so one 8-byte address per lane
// moves twice the data of the two-address forms.  Such a read must be 8-byte
// aligned, which a channel's offset (in dwords) is only when it is even.  For
// an odd offset m the read starts one dword early, at m - 1: its second
// dword is the lane's first (added to e0 as for even offsets) and its first
// dword is lane l - 1's second, so it goes to a third set of sums, od, which
// is moved one lane down when the packed sums are widened (every 256
// channels: `wave_shl` DPP, lane 63 taking the next block's lane 0).  The
// last block's lane 63 has no right neighbour: lane j reads that dword for
// channel j once per channel group, and the wave's total is added at the end.
// The offsets' parities are wave-uniform, so each pair of channels takes one
// of four branches, in which equal targets still share a 3-input add.  The
// LDS offset of each channel for the wave's DM is computed once per group by
// lane j for channel j and broadcast with readlane.
//
// Subband dedispersion runs on the same kernel.  Step one is a grouped job:
// every subband is an independent problem over its own channels, and its sums
// are stored as uint16.  Step two treats the subbands as channels and the
// fine DMs of one coarse DM as the DM trials, again one group per coarse DM;
// its uint16 input is staged as is (no widening) and its packed 16-bit sums
// are widened every `flush_every` subbands, before they can overflow.
#include "internal.h"

#include <cstdlib>

namespace amber {
namespace {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// acc += a (+ b) as one VALU instruction the compiler cannot merge with
// others (plain adds in the branches of a switch get their common part moved
// behind it).
__device__ __forceinline__ void add_to(uint32_t &acc, uint32_t a)
{
    asm("v_add_u32 %0, %1, %0" : "+v"(acc) : "v"(a));
}
__device__ __forceinline__ void add3_to(uint32_t &acc, uint32_t a, uint32_t b)
{
    asm("v_add3_u32 %0, %1, %2, %0" : "+v"(acc) : "v"(a), "v"(b));
}

// Sum over the wavefront (every lane gets it): DPP within rows of 16, then
// across rows through readlane.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, true);   // quad_perm [1,0,3,2]
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, true);   // quad_perm [2,3,0,1]
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, true);  // row_half_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, true);  // row_mirror
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const u32x2 lds_u2;
typedef __attribute__((address_space(3))) u32x4 lds_w4;
typedef __attribute__((address_space(3))) const uint32_t lds_u1;

// v_perm_b32 selector that widens bytes a and a + 1 of {hi, lo} into the two
// 16-bit halves of a dword (selector byte 0x0c yields zero).
__host__ __device__ constexpr uint32_t widen_sel(int a)
{
    return (uint32_t)a | 0x0c00u | ((uint32_t)(a + 1) << 16) | 0x0c000000u;
}

// Maps the round-robin dispatch of work-groups over the 8 XCDs onto tiles so
// that the groups one XCD runs are consecutive DM blocks of the same time tile
// and share their input windows in that XCD's L2.
__device__ __forceinline__ void tile_of_block(int id, int nx, int ny, int remap, int &tx, int &ty)
{
    if (remap) {
        const int nb = nx * ny;
        const int xcd = id & 7, local = id >> 3;
        const int per = nb >> 3, rem = nb & 7;
        const int logical = xcd * per + (xcd < rem ? xcd : rem) + local;
        ty = logical % ny;
        tx = logical / ny;
    } else {
        tx = id % nx;
        ty = id / nx;
    }
}

struct StageArgs {
    const uint8_t *in;
    int64_t in_stride, in_bytes;
    const int32_t *dfirst;
    int64_t t0;
    int n_chan, items_per_row, n_items;
};

// A staging item is two chunks of 8 samples.  uint8 input: the chunks lie
// half a row apart (chunks it and it + items_per_row of its row), each loaded
// with one dword of lookahead, so that the item's writes of one chunk and
// copy cover consecutive 16-byte lines across the lanes, which reach every
// LDS bank.  uint16 input (subband step two): the chunks are adjacent (chunks
// 2 it and 2 it + 1), loaded as one piece of 16 samples and a dword of
// lookahead, the first chunk's lookahead being the second's first dword:
// three loads instead of four, which measured faster there than covering
// every bank.  `at` is the first dword of chunk 1 in the item's registers.
template <bool U16>
struct Item {
    static constexpr int at = U16 ? 4 : 3;
    static constexpr int dwords = U16 ? 9 : 6;
};

// A buffer resource over n bytes from p: loads past the end read zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t range_rsrc(const void *p, uint32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)n, 0x00020000);
}

// Per-item constants of the staging loads: byte offset of the item's first
// sample within the group's rows, apart from the first DM's delay, and the
// byte offset of the item's channel in a delay row (from the group's first).
template <bool U16, int MAXI>
struct ItemBase {
    uint32_t off[MAXI], dch[MAXI];
};

// Issues the loads of staging items tid + m * nthreads (m < MAXI) of the
// channel group starting at c0: two chunks of 8 samples + lookahead each
// (one piece of 16 for 16-bit input).  The loads are buffer loads over the
// group's rows up to the job's last channel (and the delays of those
// channels), so the hardware range check turns every dword past them (past
// the last row's samples, or an item past the last channel) into zero; no
// load sits under a branch and nothing here reads a loaded value except the
// delays, so the input loads stay in flight through the group's sums (buffer
// loads count against the vector-memory counter only: flat loads through
// generic pointers would also count against the LDS one, and every wait for
// a sum's LDS read would wait for them).  Offsets are 32-bit from the
// group's first row: the host keeps channel_unroll * in_stride below 2^32,
// and a window that runs past its row's end (or wraps, or starts before the
// buffer for a table that breaks its contract) only feeds outputs at or past
// n_out.
template <int CU, bool U16, int MAXI>
__device__ __forceinline__ void stage_load(const StageArgs &a, int c0, const ItemBase<U16, MAXI> &ib,
                                           uint32_t (&w)[MAXI][Item<U16>::dwords])
{
    const int left = a.n_chan - c0;  // channels from c0 to the job's last one
    const __amdgpu_buffer_rsrc_t rd = range_rsrc(a.dfirst + c0, left > 0 ? 4u * (uint32_t)left : 0u);
    int df[MAXI];
#pragma unroll
    for (int m = 0; m < MAXI; ++m) df[m] = __builtin_amdgcn_raw_buffer_load_b32(rd, ib.dch[m], 0, 0);
    // the range: the group's rows, not past the job's last channel (in a
    // grouped job the next group's rows follow) nor past the buffer; in 32
    // bits, as CU rows are below 2^32 bytes
    const int64_t start = (int64_t)c0 * a.in_stride;  // wave-uniform
    const int64_t rest = a.in_bytes - start;
    const uint32_t rows = left <= 0 ? 0u : (uint32_t)(left < CU ? left : CU) * (uint32_t)a.in_stride;
    const int rest_hi = (int)(rest >> 32);
    const uint32_t n = rest_hi < 0 ? 0u : (rest_hi > 0 ? rows : min((uint32_t)rest, rows));
    const __amdgpu_buffer_rsrc_t rs = range_rsrc(a.in + (n ? start : 0), n);
    const uint32_t half = 8u * (uint32_t)a.items_per_row;  // bytes between the chunks of a uint8 item
#pragma unroll
    for (int m = 0; m < MAXI; ++m) {
        // first sample of the window, rounded down to a dword boundary (t0 is
        // a multiple of 4)
        const uint32_t o = ib.off[m] + (U16 ? ((uint32_t)df[m] << 1) & ~3u : (uint32_t)df[m] & ~3u);
        uint32_t *d = w[m];
        if constexpr (U16) {
            const i32x4v v0 = __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0);
            const i32x4v v1 = __builtin_amdgcn_raw_buffer_load_b128(rs, o + 16u, 0, 0);
            d[0] = v0.x;
            d[1] = v0.y;
            d[2] = v0.z;
            d[3] = v0.w;
            d[4] = v1.x;
            d[5] = v1.y;
            d[6] = v1.z;
            d[7] = v1.w;
            d[8] = __builtin_amdgcn_raw_buffer_load_b32(rs, o + 32u, 0, 0);
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, o + (h ? half : 0u), 0, 0);
                d[3 * h] = v[0];
                d[3 * h + 1] = v[1];
                d[3 * h + 2] = v[2];
            }
        }
    }
}

// Writes staging item q (two chunks of 8 samples) as 16-bit values into the
// two copies: copy s, dword m of a chunk holds its samples 2m + s and
// 2m + s + 1.  A chunk and copy is one 16-byte line.
template <int CU, bool U16>
__device__ __forceinline__ void stage_store(lds_w4 *lds, int win2, int items_per_row, int n_items, int q,
                                            uint32_t (&w)[Item<U16>::dwords])
{
    if (q >= n_items) return;
    const int j = q / items_per_row;
    const int it = q - j * items_per_row;
    // the copy and chunk distances pass through an SGPR move the compiler
    // cannot hoist, so that the four write addresses are formed here from one
    // base instead of living in registers (or scratch) across the loop
    int copy_w4 = (CU * win2) >> 2, half_w4 = items_per_row;
    asm volatile("s_mov_b32 %0, %0" : "+s"(copy_w4));
    asm volatile("s_mov_b32 %0, %0" : "+s"(half_w4));
    if (U16) half_w4 = 1;  // adjacent chunks
    lds = lds + ((j * win2) >> 2) + (U16 ? 2 * it : it);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t *c = &w[h * Item<U16>::at];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            uint32_t d[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (U16) {  // samples 2m + s, 2m + s + 1 of the chunk's dwords
                    d[m] = s == 0 ? c[m] : __builtin_amdgcn_alignbyte(c[m + 1], c[m], 2);
                } else {
                    const int p = 2 * m + s;  // first byte of the pair within the 12 bytes
                    d[m] = __builtin_amdgcn_perm(c[(p >> 2) + 1], c[p >> 2], widen_sel(p & 3));
                }
            }
            lds[s * copy_w4 + h * half_w4] = u32x4{d[0], d[1], d[2], d[3]};
        }
    }
}

// Wavefronts per SIMD the register allocation must allow: 8 (two 1024-item
// work-groups per CU, at most 64 registers) where the kernel then spills at
// most a few registers outside the channel loop (the tiles of 4 and 8
// samples per work-item with shallow staging); elsewhere 1, i.e. no limit
// (a 1024-item work-group then has a CU to itself).
template <int M, int MAXI, bool U16, int DPT>
constexpr int waves_per_simd()
{
    if (U16) return 1;
    if (M == 2) return (MAXI <= 2 || (MAXI == 3 && DPT == 1)) ? 8 : 1;
    if (M == 4) return (MAXI == 1 || (MAXI == 2 && DPT == 1)) ? 8 : 1;
    return 1;
}

template <int M, int CU, int MAXI, bool U16, int DPT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(waves_per_simd<M, MAXI, U16, DPT>())))
void dedisperse_kernel(DedispJob single, const DedispJob *__restrict__ jobs, int n_jobs, int tpd, int dpb, int remap)
{
    static_assert(CU <= 32, "one lane per channel of a group, channel bits in 32-bit masks");
    extern __shared__ u32x4 lds_raw[];
    lds_w4 *lds = (lds_w4 *)lds_raw;

    // One job (beam) per launch, or a table of jobs whose tiles are laid out
    // back to back in the grid.
    int block = blockIdx.x;
    DedispJob job = single;
    if (jobs) {
        int j = 0;
        while (j + 1 < n_jobs && jobs[j + 1].block_start <= block) ++j;
        job = jobs[j];
        block -= job.block_start;
    }
    if (job.groups > 1) {  // independent problems of one shape, back to back in the grid
        const int gi = block / job.group_blocks;
        block -= gi * job.group_blocks;
        job.delays += gi * job.group_delays;
        job.in += gi * job.group_in;
        job.in_bytes -= gi * job.group_in;
        job.dd = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(job.dd) + gi * job.group_out);
        if (job.keep) job.keep += gi * job.group_keep;
    }
    const int32_t *__restrict__ delays = job.delays;
    const int n_dm = job.n_dm, n_chan = job.n_chan, win = job.win, omax = job.omax;
    const int64_t n_out = job.n_out, dd_stride = job.dd_stride;

    const int win2 = win >> 1;  // dwords per staged row copy
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int wave = uniform(tid >> 6);
    const int lane = tid & 63;
    const int waves_per_dm = tpd >> 6;
    const int dm_local = uniform(wave / waves_per_dm);
    const int wave_t = uniform((wave - dm_local * waves_per_dm) * 128 * M);  // first sample of the wave
    int tx, ty;
    tile_of_block(block, job.tiles_t, job.tiles_dm, remap, tx, ty);
    // the work-group's DMs: dpb wave slots of DPT consecutive DMs each
    const int i0 = ty * dpb * DPT;
    const int i = i0 + dm_local * DPT;  // the wave's first DM
    const bool active = i < n_dm;
    const int64_t t0 = (int64_t)tx * tpd * 2 * M;

    StageArgs sa;
    sa.in = job.in;
    sa.in_stride = job.in_stride;
    sa.in_bytes = job.in_bytes;
    sa.dfirst = delays + (size_t)i0 * n_chan;
    sa.t0 = t0;
    sa.n_chan = n_chan;
    sa.items_per_row = win >> 4;
    sa.n_items = CU * sa.items_per_row;
    // delay rows of the wave's DMs (rows past n_dm read the first DM's row;
    // their sums are never stored)
    const int32_t *dmine[DPT];
#pragma unroll
    for (int r = 0; r < DPT; ++r) dmine[r] = delays + (size_t)(i + r < n_dm ? i + r : i0) * n_chan;

    // Packed 16-bit sums per DM and 128-dword block k of the wave's outputs
    // (lane l owns dwords 2l and 2l + 1 of each block): e0 / e1 the block's
    // first / second dword of the lane from even-aligned reads, od the first
    // dword of odd-aligned reads (it belongs to lane l - 1's second dword).
    // lo0/hi0/lo1/hi1: the widened 32-bit totals of the lane's four samples.
    constexpr int K = M / 2;
    static_assert(M % 2 == 0, "whole 8-byte reads per lane");
    uint32_t e0[DPT][K], e1[DPT][K], od[DPT][K];
    uint32_t lo0[DPT][K], hi0[DPT][K], lo1[DPT][K], hi1[DPT][K];
    // the last block's lane 63 second dword from odd-aligned reads: summed
    // per channel by lane j, and added to lane 63's totals over the wave.
    // uint8 input: packed sums fx, summed over the wave at each widening
    // (every 256 channels).  uint16 input, whose packed sums are widened
    // every few channels: 32-bit halves fxl / fxh summed over the wave once
    // at the end, and likewise the od sums widened in place (odl / odh) and
    // moved one lane down once at the end, not at every widening.
    uint32_t fx[DPT], fxl[DPT], fxh[DPT];
    uint32_t odl[DPT][K], odh[DPT][K];
#pragma unroll
    for (int r = 0; r < DPT; ++r) {
        fx[r] = fxl[r] = fxh[r] = 0u;
#pragma unroll
        for (int k = 0; k < K; ++k) odl[r][k] = odh[r][k] = 0u;
#pragma unroll
        for (int k = 0; k < K; ++k) e0[r][k] = e1[r][k] = od[r][k] = lo0[r][k] = hi0[r][k] = lo1[r][k] = hi1[r][k] = 0u;
    }

    // Prefetch of the first channel group: input items, and on lane j < CU the
    // delays of channel j for this wave's DM and for the group's first DM.
    ItemBase<U16, MAXI> ib;
#pragma unroll
    for (int m = 0; m < MAXI; ++m) {
        const int q = tid + m * nthreads;
        const int j = q / sa.items_per_row;
        const int it = q - j * sa.items_per_row;
        // (an item past the last one, never stored, may wrap: its loads stay
        // range-checked)
        ib.off[m] = (uint32_t)j * (uint32_t)sa.in_stride + (U16 ? 2u * ((uint32_t)t0 + 16u * (uint32_t)it)
                                                               : (uint32_t)t0 + 8u * (uint32_t)it);
        ib.dch[m] = 4u * (uint32_t)j;
    }
    uint32_t pre[MAXI][Item<U16>::dwords];
    stage_load<CU, U16, MAXI>(sa, 0, ib, pre);
    const int cl = lane < CU ? lane : CU - 1;
    // Zapped channels (keep flag 0) are staged like any other; their offsets
    // are redirected to a zeroed LDS region of 64 * M dwords after the two
    // copies, so they add nothing.  The flag is loaded once per channel group
    // beside the delays: a test inside the staging loads would serialise them.
    const uint8_t *__restrict__ keep = job.keep;
    const uint32_t zero_off = 4u * (uint32_t)(2 * CU * win2);
    if (keep) {
        uint32_t *zl = (uint32_t *)lds_raw + 2 * CU * win2;
        for (int q = tid; q < 64 * M; q += nthreads) zl[q] = 0u;
    }
    // keep flags are read unconditionally (from the delay table when there
    // are none) so that no load sits under a branch
    // Delays (and keep flags) of channel c0 + lane for the group at c0:
    // buffer loads over the rest of each row, zero past the last channel (a
    // channel there is staged from zeros, so any offset in range adds nothing).
    const uint8_t *kp = keep ? keep : reinterpret_cast<const uint8_t *>(delays);
    int d_next[DPT], f_next = 0, k_next = 1;
    const uint32_t lane_off = 8u * (uint32_t)lane;
    auto load_delays = [&](int c) {
        const uint32_t lane4 = lane_off >> 1;
        const uint32_t rest = c < n_chan ? (uint32_t)(n_chan - c) : 0u;
#pragma unroll
        for (int r = 0; r < DPT; ++r)
            d_next[r] = __builtin_amdgcn_raw_buffer_load_b32(range_rsrc(dmine[r] + c, 4u * rest), lane4, 0, 0);
        f_next = __builtin_amdgcn_raw_buffer_load_b32(range_rsrc(sa.dfirst + c, 4u * rest), lane4, 0, 0);
        k_next = __builtin_amdgcn_raw_buffer_load_b8(range_rsrc(kp + c, keep ? rest : 0u), (uint32_t)lane, 0, 0);
    };
    load_delays(0);
    // LDS byte offset of channel cl's window at offset 0 in copy 0 for this
    // wave, and the distance to copy 1 (its dword count is a multiple of 8)
    const uint32_t lane_base = 4u * (uint32_t)(cl * win2 + (wave_t >> 1));
    const uint32_t copy1 = 4u * (uint32_t)(CU * win2);

    const __attribute__((address_space(3))) char *ldsb = (const __attribute__((address_space(3))) char *)lds;

    // Moves the packed sums into the 32-bit totals.  A lane's second dword
    // from odd-aligned reads is its right neighbour's od (lane 63: the next
    // block's lane 0; for the last block it is the fx term).
    auto widen = [&]() {
        if constexpr (U16) {
#pragma unroll
            for (int r = 0; r < DPT; ++r)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    lo0[r][k] += e0[r][k] & 0xffffu;
                    hi0[r][k] += e0[r][k] >> 16;
                    lo1[r][k] += e1[r][k] & 0xffffu;
                    hi1[r][k] += e1[r][k] >> 16;
                    odl[r][k] += od[r][k] & 0xffffu;
                    odh[r][k] += od[r][k] >> 16;
                    e0[r][k] = e1[r][k] = od[r][k] = 0u;
                }
            return;
        }
#pragma unroll
        for (int r = 0; r < DPT; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t nxt = k + 1 < K ? (uint32_t)__builtin_amdgcn_readlane((int)od[r][k + 1], 0) : 0u;
                // wave_shl:1, lane 63 keeps `nxt`
                const uint32_t os = (uint32_t)__builtin_amdgcn_update_dpp((int)nxt, (int)od[r][k], 0x130, 0xf, 0xf,
                                                                          false);
                lo0[r][k] += e0[r][k] & 0xffffu;
                hi0[r][k] += e0[r][k] >> 16;
                lo1[r][k] += (e1[r][k] & 0xffffu) + (os & 0xffffu);
                hi1[r][k] += (e1[r][k] >> 16) + (os >> 16);
                e0[r][k] = e1[r][k] = od[r][k] = 0u;
            }
#pragma unroll
        for (int r = 0; r < DPT; ++r) {
            const uint32_t slo = wave_sum_u32(fx[r] & 0xffffu), shi = wave_sum_u32(fx[r] >> 16);
            if (lane == 63) {
                lo1[r][K - 1] += slo;
                hi1[r][K - 1] += shi;
            }
            fx[r] = 0u;
        }
    };

    int since_flush = 0;
    const int flush_every = U16 ? uniform(job.flush_every) : 256;
    int left = flush_every;  // channels the packed sums may still take (uint16 input)
    for (int c0 = 0; c0 < n_chan; c0 += CU) {
#pragma unroll
        for (int m = 0; m < MAXI; ++m)
            stage_store<CU, U16>(lds, win2, sa.items_per_row, sa.n_items, tid + m * nthreads, pre[m]);
        // LDS byte offset of channel `cl` for each of this wave's DMs, rounded
        // down to 8 bytes, and whether it was odd in dwords (the wave's reads
        // then start one dword early)
        uint32_t chan_al[DPT];
        uint32_t par[DPT];   // bit j: channel j is odd (CU <= 32 on this path's instantiations)
        bool odd_l[DPT];     // this lane's channel is odd
        const int fa = (f_next & (U16 ? 1 : 3)) - f_next;
        const bool zap = keep && k_next == 0;
        const bool mine = !zap && lane < CU;
#pragma unroll
        for (int r = 0; r < DPT; ++r) {
            const int oo = d_next[r] + fa;
            const int o = min(max(oo, 0), omax);
            // copy o & 1, dword o >> 1: rounded down to 8 bytes, and whether
            // the dword was odd
            const uint32_t h = (uint32_t)o >> 1;
            const uint32_t cb = lane_base + ((uint32_t)o & 1u) * copy1;
            chan_al[r] = zap ? zero_off : cb + 4u * (h & ~1u);
            odd_l[r] = mine && (h & 1u);
            par[r] = (uint32_t)__builtin_amdgcn_ballot_w64(odd_l[r]);
        }
        __syncthreads();
        // Prefetch of the next group, also after the last one (its items are
        // all invalid and read one shared address): a branch here would make
        // the compiler copy the loaded registers at its join and so wait for
        // the loads before the sums.
        stage_load<CU, U16, MAXI>(sa, c0 + CU, ib, pre);
        load_delays(c0 + CU);

        if (active) {
            // the last block's lane 63 second dword of the odd channels: lane j
            // reads it for channel j (the dword after the wave's reads)
#pragma unroll
            for (int r = 0; r < DPT; ++r) {
                // (even lanes read a dword of the window they never use: the
                // address stays in range)
                const bool odd = odd_l[r];
                const uint32_t v = *(lds_u1 *)(ldsb + (odd ? chan_al[r] : 0u) + 512u * K);
                if constexpr (U16) {
                    fxl[r] += odd ? (v & 0xffffu) : 0u;
                    fxh[r] += odd ? (v >> 16) : 0u;
                } else {
                    fx[r] += odd ? v : 0u;
                }
            }
            if constexpr (!U16 && CU >= 2) {
                // channel pairs: one branch on both channels' alignment, so
                // that equal targets still take one 3-input add
#pragma unroll
                for (int j = 0; j < CU; j += 2) {
#pragma unroll
                    for (int r = 0; r < DPT; ++r) {
                        const uint32_t ba = (uint32_t)__builtin_amdgcn_readlane((int)chan_al[r], j);
                        const uint32_t bb = (uint32_t)__builtin_amdgcn_readlane((int)chan_al[r], j + 1);
                        lds_u2 *pa = (lds_u2 *)(ldsb + (ba + lane_off));
                        lds_u2 *pb = (lds_u2 *)(ldsb + (bb + lane_off));
                        u32x2 xa[K], xb[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            // one 8-byte address per lane and read: kept apart, the
                            // compiler would pair the blocks into a two-address read
                            xa[k] = pa[64 * k];
                            xb[k] = pb[64 * k];
                            asm volatile("" ::: "memory");
                        }
                        // (the adds are written as single instructions so that
                        // the compiler cannot move the cases' common "e0 +="
                        // behind the branch, which would cost one more add)
                        const uint32_t cls = uniform((int)((par[r] >> j) & 3u));
                        if (cls == 0u) {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                add3_to(e0[r][k], xa[k].x, xb[k].x);
                                add3_to(e1[r][k], xa[k].y, xb[k].y);
                            }
                        } else if (cls == 3u) {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                add3_to(e0[r][k], xa[k].y, xb[k].y);
                                add3_to(od[r][k], xa[k].x, xb[k].x);
                            }
                        } else if (cls == 1u) {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                add3_to(e0[r][k], xa[k].y, xb[k].x);
                                add_to(e1[r][k], xb[k].y);
                                add_to(od[r][k], xa[k].x);
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                add3_to(e0[r][k], xa[k].x, xb[k].y);
                                add_to(e1[r][k], xa[k].y);
                                add_to(od[r][k], xb[k].x);
                            }
                        }
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < CU; ++j) {
#pragma unroll
                    for (int r = 0; r < DPT; ++r) {
                        const uint32_t ba = (uint32_t)__builtin_amdgcn_readlane((int)chan_al[r], j);
                        lds_u2 *pa = (lds_u2 *)(ldsb + (ba + lane_off));
                        u32x2 xa[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            xa[k] = pa[64 * k];
                            asm volatile("" ::: "memory");
                        }
                        if (uniform((int)((par[r] >> j) & 1u)) == 0) {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                add_to(e0[r][k], xa[k].x);
                                add_to(e1[r][k], xa[k].y);
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                add_to(e0[r][k], xa[k].y);
                                add_to(od[r][k], xa[k].x);
                            }
                        }
                    }
                    if (U16 && --left == 0) {
                        widen();
                        left = flush_every;
                    }
                }
            }
            since_flush += CU;
            if ((!U16 && since_flush >= 256) || c0 + CU >= n_chan) {
                widen();
                since_flush = 0;
            }
        }
        __syncthreads();
    }

    if (!active) return;
    if constexpr (U16) {
        // the od totals one lane down (lane 63: the next block's lane 0; for
        // the last block the fx terms summed over the wave)
#pragma unroll
        for (int r = 0; r < DPT; ++r) {
            const uint32_t slo = wave_sum_u32(fxl[r]), shi = wave_sum_u32(fxh[r]);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t nl = k + 1 < K ? (uint32_t)__builtin_amdgcn_readlane((int)odl[r][k + 1], 0) : slo;
                const uint32_t nh = k + 1 < K ? (uint32_t)__builtin_amdgcn_readlane((int)odh[r][k + 1], 0) : shi;
                lo1[r][k] += (uint32_t)__builtin_amdgcn_update_dpp((int)nl, (int)odl[r][k], 0x130, 0xf, 0xf, false);
                hi1[r][k] += (uint32_t)__builtin_amdgcn_update_dpp((int)nh, (int)odh[r][k], 0x130, 0xf, 0xf, false);
            }
        }
    }
    const int store_vec = job.store_vec;
#pragma unroll
    for (int r = 0; r < DPT; ++r) {
        if (i + r >= n_dm) break;
        if (job.out_u16) {  // sums known to fit 16 bits: one dword per sample pair
            uint16_t *__restrict__ out =
                reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(job.dd) + (size_t)(i + r) * dd_stride * 2);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t t = t0 + wave_t + 256 * k + 4 * lane;
                const uint32_t v[4] = {lo0[r][k], hi0[r][k], lo1[r][k], hi1[r][k]};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int64_t th = t + 2 * h;
                    if (store_vec && th + 2 <= n_out) {
                        *reinterpret_cast<uint32_t *>(out + th) = v[2 * h] | (v[2 * h + 1] << 16);
                    } else {
                        if (th < n_out) out[th] = (uint16_t)v[2 * h];
                        if (th + 1 < n_out) out[th + 1] = (uint16_t)v[2 * h + 1];
                    }
                }
            }
        } else {
            int32_t *__restrict__ out = job.dd + (size_t)(i + r) * dd_stride;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t t = t0 + wave_t + 256 * k + 4 * lane;
                const uint32_t v[4] = {lo0[r][k], hi0[r][k], lo1[r][k], hi1[r][k]};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int64_t th = t + 2 * h;
                    if (store_vec && th + 2 <= n_out) {
                        *reinterpret_cast<int2 *>(out + th) = make_int2((int)v[2 * h], (int)v[2 * h + 1]);
                    } else {
                        if (th < n_out) out[th] = (int32_t)v[2 * h];
                        if (th + 1 < n_out) out[th + 1] = (int32_t)v[2 * h + 1];
                    }
                }
            }
        }
    }
}

using KernelFn = void (*)(DedispJob, const DedispJob *, int, int, int, int);

// uint8 input: every (samples_per_thread, channel_unroll) with the staging
// depths the planner allows (4 below 16 samples per work-item, 3 at 16, 2 at
// 32), one DM per wavefront; two DMs per wavefront up to 16 samples per
// work-item (staging depth 2 at 16).  uint16 input (subband step two, at most a few dozen subbands):
// 8 or 16 samples per work-item, channel_unroll 4..32, staging depth 1..2,
// one DM per wavefront.  Deeper staging would not fit the 128 registers of a
// 1024-item work-group.
template <int M, int CU, bool U16, int DPT>
KernelFn pick_items(int maxi)
{
    constexpr int cap = U16 ? 2 : (M >= 16 ? 2 : (M >= 8 ? (DPT == 2 ? 2 : 3) : 4));
    switch (maxi) {
    case 1: return dedisperse_kernel<M, CU, 1, U16, DPT>;
    case 2: return dedisperse_kernel<M, CU, 2, U16, DPT>;
    case 3:
        if constexpr (cap >= 3) return dedisperse_kernel<M, CU, 3, U16, DPT>;
        return nullptr;
    case 4:
        if constexpr (cap >= 4) return dedisperse_kernel<M, CU, 4, U16, DPT>;
        return nullptr;
    }
    return nullptr;
}

template <int M, int DPT>
KernelFn pick_cu(int cu, int maxi, int u16)
{
    if (u16) {
        if constexpr ((M == 4 || M == 8) && DPT == 1) {
            switch (cu) {
            case 4: return pick_items<M, 4, true, 1>(maxi);
            case 8: return pick_items<M, 8, true, 1>(maxi);
            case 16: return pick_items<M, 16, true, 1>(maxi);
            case 32: return pick_items<M, 32, true, 1>(maxi);
            }
        }
        return nullptr;
    }
    if constexpr (DPT == 1 || M <= 8) {
        switch (cu) {
        case 1: return pick_items<M, 1, false, DPT>(maxi);
        case 2: return pick_items<M, 2, false, DPT>(maxi);
        case 4: return pick_items<M, 4, false, DPT>(maxi);
        case 8: return pick_items<M, 8, false, DPT>(maxi);
        case 16: return pick_items<M, 16, false, DPT>(maxi);
        case 32: return pick_items<M, 32, false, DPT>(maxi);
        }
    }
    return nullptr;
}

template <int DPT>
KernelFn pick_spt(int spt, int cu, int maxi, int u16)
{
    switch (spt) {
    case 4: return pick_cu<2, DPT>(cu, maxi, u16);
    case 8: return pick_cu<4, DPT>(cu, maxi, u16);
    case 16: return pick_cu<8, DPT>(cu, maxi, u16);
    case 32: return pick_cu<16, DPT>(cu, maxi, u16);
    }
    return nullptr;
}

KernelFn pick(int spt, int cu, int maxi, int u16, int dpt)
{
    switch (dpt) {
    case 1: return pick_spt<1>(spt, cu, maxi, u16);
    case 2: return pick_spt<2>(spt, cu, maxi, u16);
    }
    return nullptr;
}

int xcd_remap_setting()
{
    const char *e = getenv("AMBER_XCD_REMAP");
    return e ? atoi(e) : 1;
}

}  // namespace

amber_status check_stage_stride(const DedispPlan &p, int64_t in_stride)
{
    if (!p.direct && (int64_t)p.cu * in_stride > kMaxStageSpan)
        return fail(AMBER_E_SHAPE, "channel_unroll %d x input row stride %lld bytes exceeds 2^32 (the staged "
                    "kernel's offsets within a channel group)", p.cu, (long long)in_stride);
    return AMBER_OK;
}

DedispJob make_dedisp_job(const DedispPlan &p, const int32_t *d_delays, int n_dm, int n_chan, const uint8_t *d_in,
                          int64_t in_stride, int32_t *d_dd, int64_t dd_stride, int64_t n_out)
{
    DedispJob j{};
    j.delays = d_delays;
    j.in = d_in;
    j.dd = d_dd;
    j.in_stride = in_stride;
    j.in_bytes = (int64_t)n_chan * in_stride;
    j.dd_stride = dd_stride;
    j.n_out = n_out;
    j.n_dm = n_dm;
    j.n_chan = n_chan;
    j.win = p.win;
    j.omax = p.omax;
    j.tiles_t = (int)((n_out + p.tile_t - 1) / p.tile_t);
    j.tiles_dm = (n_dm + p.dpb * p.dpt - 1) / (p.dpb * p.dpt);
    j.store_vec = (dd_stride % 2 == 0) && (((uintptr_t)d_dd & 7) == 0);
    j.block_start = 0;
    j.flush_every = 256;
    j.groups = 1;
    return j;
}

amber_status launch_dedisperse_jobs(const DedispPlan &p, const DedispJob *single, const DedispJob *d_jobs,
                                    int n_jobs, int64_t n_blocks, int64_t lds_bytes, hipStream_t stream)
{
    KernelFn fn = pick(p.spt, p.cu, p.maxi, p.in_u16, p.dpt);
    if (!fn)
        return fail(AMBER_E_CONFIG, "no dedispersion kernel for spt=%d cu=%d maxi=%d dpt=%d%s", p.spt, p.cu, p.maxi,
                    p.dpt, p.in_u16 ? " with 16-bit input (spt 8 or 16, channel_unroll 4..32, 1 DM per wave)" : "");
    if (lds_bytes > 64 * 1024)
        AMBER_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes),
                  "hipFuncSetAttribute(dedisperse)");
    if (n_blocks > 0x7fffffff) return fail(AMBER_E_SHAPE, "grid of %lld work-groups is too large", (long long)n_blocks);
    static const int remap = xcd_remap_setting();
    hipLaunchKernelGGL(fn, dim3((unsigned)n_blocks), dim3(p.threads), (size_t)lds_bytes, stream,
                       single ? *single : DedispJob{}, d_jobs, n_jobs, p.tpd, p.dpb, d_jobs ? 0 : remap);
    AMBER_HIP(hipGetLastError(), "dedisperse launch");
    return AMBER_OK;
}

amber_status launch_dedisperse(const DedispPlan &p, const int32_t *d_delays, int n_dm, int n_chan,
                               const uint8_t *d_in, int64_t in_stride, int64_t n_in, int32_t *d_dd,
                               int64_t dd_stride, int64_t n_out, hipStream_t stream, const uint8_t *d_keep)
{
    (void)n_in;
    DedispJob j = make_dedisp_job(p, d_delays, n_dm, n_chan, d_in, in_stride, d_dd, dd_stride, n_out);
    j.keep = d_keep;
    const int64_t lds = p.lds_bytes + (d_keep ? mask_lds_bytes(p) : 0);
    if (lds > kMaxLdsBytes)
        return fail(AMBER_E_CONFIG, "masked dedispersion tile needs %lld B of LDS (limit %lld)", (long long)lds,
                    (long long)kMaxLdsBytes);
    return launch_dedisperse_jobs(p, &j, nullptr, 1, (int64_t)j.tiles_t * j.tiles_dm, lds, stream);
}

}  // namespace amber
