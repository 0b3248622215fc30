// Issue-rate and bandwidth microbenchmarks of gfx950 that the roofline peaks
// of the search kernels rest on: 32-bit integer VALU forms (one add, three-
// operand add, packed 16-bit add), the FP64 forms of the S/N moments, LDS
// reads of every width the kernels use, and a device-memory copy.
//
// Every kernel runs `iters` loop trips of a fixed body; the host entry point
// times one launch with HIP events and reports the operations (or bytes) of
// the launch per second.  The VALU bodies keep 8 independent chains per
// work-item so that issue, not latency, bounds them; the LDS bodies read a
// conflict-free pattern (consecutive lanes, consecutive 4/8/16-byte words)
// from a 64 KiB array and fold the words with three-operand adds.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

#define CHAINS 8

template <int KIND>
__global__ __launch_bounds__(256) void valu_kernel(uint32_t *out, uint32_t seed, int iters)
{
    uint32_t a[CHAINS];
    double f[CHAINS];
    uint64_t u[CHAINS];
    float g[CHAINS];
    const uint32_t b = seed ^ blockIdx.x, c = seed * 3u + threadIdx.x;
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) {
        a[j] = threadIdx.x * 7u + j * seed;
        f[j] = (double)a[j];
        u[j] = a[j];
        g[j] = 0.f;
    }
    const double fb = (double)b * 1e-9;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < CHAINS; ++j) {
            if (KIND == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            if (KIND == 1) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
            if (KIND == 2) asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            if (KIND == 3) asm volatile("v_lshl_or_b32 %0, %0, 4, %1" : "+v"(a[j]) : "v"(b));
            if (KIND == 4) asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(f[j]) : "v"(fb));
            if (KIND == 5) asm volatile("v_cvt_f64_i32 %0, %1" : "=v"(f[j]) : "v"(a[j] + (uint32_t)i));
            if (KIND == 6) asm volatile("v_max3_i32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
            if (KIND == 7) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(u[j]) : "v"(a[j]), "v"(b) : "vcc");
            if (KIND == 8) asm volatile("v_add_f64 %0, %0, %1" : "+v"(f[j]) : "v"(fb));
            if (KIND == 9) asm volatile("v_max_f64 %0, %0, %1" : "+v"(f[j]) : "v"(fb));
            if (KIND == 10) asm volatile("v_cvt_f32_i32 %0, %1" : "=v"(g[j]) : "v"(a[j] + (uint32_t)i));
            if (KIND == 11) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            if (KIND == 12) asm volatile("v_cvt_f64_u32 %0, %1" : "=v"(f[j]) : "v"(a[j] + (uint32_t)i));
            if (KIND == 13) asm volatile("v_sub_u32 %0, %1, %0" : "+v"(a[j]) : "v"(b));
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) s ^= a[j] ^ (uint32_t)f[j] ^ (uint32_t)u[j] ^ (uint32_t)g[j];
    if (s == 0x9e3779b9u) out[blockIdx.x] = s;
}

// LDS reads of one form per kernel: 0 ds_read_b32, 1 ds_read2st64_b32,
// 2 ds_read_b64, 3 ds_read2st64_b64, 4 ds_read_b128, 5 ds_read2_b32 of two
// adjacent dwords at an 8-byte-aligned address, 6 the same 4 bytes further
// (dwords 1 and 2 of the lane's 8-byte slot, so the pair straddles two
// slots), 7 forms 2 and 6 alternating.  One asm block per loop trip issues
// reads of 64 bytes per lane in total (16 x b32, 8 x read2st64_b32, 8 x
// b64, 4 x read2st64_b64, 4 x b128 or 8 x read2_b32) and waits for them
// before its outputs are used; lane l reads the words at byte 4 W l of each
// 256 W-byte block (W = dwords per read), so consecutive lanes touch
// consecutive words.  The 4 KiB a wave reads per trip move with the trip
// inside a 16 KiB window of the array; forms 6 and 7 read up to 4 bytes past
// the window, which the array's 16 extra bytes hold (small enough for 32
// waves per CU).
template <int FORM>
__global__ __launch_bounds__(256) void lds_kernel(uint32_t *out, int iters)
{
    constexpr int N = 4096;  // dwords, 16 KiB read window
    __shared__ __attribute__((aligned(16))) uint32_t s[N + 4];
    for (int i = threadIdx.x; i < N + 4; i += blockDim.x) s[i] = (uint32_t)i * 2654435761u;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t lds0 = (uint32_t)reinterpret_cast<uintptr_t>(s);
    constexpr int W = (FORM == 0 || FORM == 1) ? 1 : (FORM == 4 ? 4 : 2);
    static_assert(FORM >= 0 && FORM <= 7, "read form");
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
        const uint32_t addr = lds0 + ((((uint32_t)(i + wave) * 4096u) & (uint32_t)(4 * N - 1)) + 4u * W * lane);
        if (FORM == 0) {
            uint32_t r0, r1, r2, r3, r4, r5, r6, r7, r8, r9, r10, r11, r12, r13, r14, r15;
            asm volatile("ds_read_b32 %0, %16 offset:0\n\tds_read_b32 %1, %16 offset:256\n\tds_read_b32 %2, %16 offset:512\n\tds_read_b32 %3, %16 offset:768\n\tds_read_b32 %4, %16 offset:1024\n\tds_read_b32 %5, %16 offset:1280\n\tds_read_b32 %6, %16 offset:1536\n\tds_read_b32 %7, %16 offset:1792\n\tds_read_b32 %8, %16 offset:2048\n\tds_read_b32 %9, %16 offset:2304\n\tds_read_b32 %10, %16 offset:2560\n\tds_read_b32 %11, %16 offset:2816\n\tds_read_b32 %12, %16 offset:3072\n\tds_read_b32 %13, %16 offset:3328\n\tds_read_b32 %14, %16 offset:3584\n\tds_read_b32 %15, %16 offset:3840\n\ts_waitcnt lgkmcnt(0)"
                         : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7), "=&v"(r8), "=&v"(r9), "=&v"(r10), "=&v"(r11), "=&v"(r12), "=&v"(r13), "=&v"(r14), "=&v"(r15)
                         : "v"(addr));
            acc ^= (r0) ^ (r1) ^ (r2) ^ (r3) ^ (r4) ^ (r5) ^ (r6) ^ (r7) ^ (r8) ^ (r9) ^ (r10) ^ (r11) ^ (r12) ^ (r13) ^ (r14) ^ (r15);
        }
        if (FORM == 1) {
            uint2 r0, r1, r2, r3, r4, r5, r6, r7;
            asm volatile("ds_read2st64_b32 %0, %8 offset0:0 offset1:1\n\tds_read2st64_b32 %1, %8 offset0:2 offset1:3\n\tds_read2st64_b32 %2, %8 offset0:4 offset1:5\n\tds_read2st64_b32 %3, %8 offset0:6 offset1:7\n\tds_read2st64_b32 %4, %8 offset0:8 offset1:9\n\tds_read2st64_b32 %5, %8 offset0:10 offset1:11\n\tds_read2st64_b32 %6, %8 offset0:12 offset1:13\n\tds_read2st64_b32 %7, %8 offset0:14 offset1:15\n\ts_waitcnt lgkmcnt(0)"
                         : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7)
                         : "v"(addr));
            acc ^= (r0.x + r0.y) ^ (r1.x + r1.y) ^ (r2.x + r2.y) ^ (r3.x + r3.y) ^ (r4.x + r4.y) ^ (r5.x + r5.y) ^ (r6.x + r6.y) ^ (r7.x + r7.y);
        }
        if (FORM == 2) {
            uint2 r0, r1, r2, r3, r4, r5, r6, r7;
            asm volatile("ds_read_b64 %0, %8 offset:0\n\tds_read_b64 %1, %8 offset:512\n\tds_read_b64 %2, %8 offset:1024\n\tds_read_b64 %3, %8 offset:1536\n\tds_read_b64 %4, %8 offset:2048\n\tds_read_b64 %5, %8 offset:2560\n\tds_read_b64 %6, %8 offset:3072\n\tds_read_b64 %7, %8 offset:3584\n\ts_waitcnt lgkmcnt(0)"
                         : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7)
                         : "v"(addr));
            acc ^= (r0.x + r0.y) ^ (r1.x + r1.y) ^ (r2.x + r2.y) ^ (r3.x + r3.y) ^ (r4.x + r4.y) ^ (r5.x + r5.y) ^ (r6.x + r6.y) ^ (r7.x + r7.y);
        }
        if (FORM == 3) {
            uint4 r0, r1, r2, r3;
            asm volatile("ds_read2st64_b64 %0, %4 offset0:0 offset1:1\n\tds_read2st64_b64 %1, %4 offset0:2 offset1:3\n\tds_read2st64_b64 %2, %4 offset0:4 offset1:5\n\tds_read2st64_b64 %3, %4 offset0:6 offset1:7\n\ts_waitcnt lgkmcnt(0)"
                         : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
                         : "v"(addr));
            acc ^= (r0.x + r0.y + r0.z + r0.w) ^ (r1.x + r1.y + r1.z + r1.w) ^ (r2.x + r2.y + r2.z + r2.w) ^ (r3.x + r3.y + r3.z + r3.w);
        }
        if (FORM == 4) {
            uint4 r0, r1, r2, r3;
            asm volatile("ds_read_b128 %0, %4 offset:0\n\tds_read_b128 %1, %4 offset:1024\n\tds_read_b128 %2, %4 offset:2048\n\tds_read_b128 %3, %4 offset:3072\n\ts_waitcnt lgkmcnt(0)"
                         : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
                         : "v"(addr));
            acc ^= (r0.x + r0.y + r0.z + r0.w) ^ (r1.x + r1.y + r1.z + r1.w) ^ (r2.x + r2.y + r2.z + r2.w) ^ (r3.x + r3.y + r3.z + r3.w);
        }
        if (FORM >= 5) {
            // read2_b32 offsets are in dwords (at most 255), so each read
            // gets its own address register
            const uint32_t a0 = addr, a1 = addr + 512, a2 = addr + 1024, a3 = addr + 1536, a4 = addr + 2048,
                           a5 = addr + 2560, a6 = addr + 3072, a7 = addr + 3584;
            uint2 r0, r1, r2, r3, r4, r5, r6, r7;
            if (FORM == 5)
                asm volatile("ds_read2_b32 %0, %8 offset0:0 offset1:1\n\tds_read2_b32 %1, %9 offset0:0 offset1:1\n\tds_read2_b32 %2, %10 offset0:0 offset1:1\n\tds_read2_b32 %3, %11 offset0:0 offset1:1\n\tds_read2_b32 %4, %12 offset0:0 offset1:1\n\tds_read2_b32 %5, %13 offset0:0 offset1:1\n\tds_read2_b32 %6, %14 offset0:0 offset1:1\n\tds_read2_b32 %7, %15 offset0:0 offset1:1\n\ts_waitcnt lgkmcnt(0)"
                             : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7)
                             : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "v"(a5), "v"(a6), "v"(a7));
            if (FORM == 6)
                asm volatile("ds_read2_b32 %0, %8 offset0:1 offset1:2\n\tds_read2_b32 %1, %9 offset0:1 offset1:2\n\tds_read2_b32 %2, %10 offset0:1 offset1:2\n\tds_read2_b32 %3, %11 offset0:1 offset1:2\n\tds_read2_b32 %4, %12 offset0:1 offset1:2\n\tds_read2_b32 %5, %13 offset0:1 offset1:2\n\tds_read2_b32 %6, %14 offset0:1 offset1:2\n\tds_read2_b32 %7, %15 offset0:1 offset1:2\n\ts_waitcnt lgkmcnt(0)"
                             : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7)
                             : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "v"(a5), "v"(a6), "v"(a7));
            if (FORM == 7)
                asm volatile("ds_read_b64 %0, %8\n\tds_read2_b32 %1, %9 offset0:1 offset1:2\n\tds_read_b64 %2, %10\n\tds_read2_b32 %3, %11 offset0:1 offset1:2\n\tds_read_b64 %4, %12\n\tds_read2_b32 %5, %13 offset0:1 offset1:2\n\tds_read_b64 %6, %14\n\tds_read2_b32 %7, %15 offset0:1 offset1:2\n\ts_waitcnt lgkmcnt(0)"
                             : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7)
                             : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "v"(a5), "v"(a6), "v"(a7));
            acc ^= (r0.x + r0.y) ^ (r1.x + r1.y) ^ (r2.x + r2.y) ^ (r3.x + r3.y) ^ (r4.x + r4.y) ^ (r5.x + r5.y) ^ (r6.x + r6.y) ^ (r7.x + r7.y);
        }
    }
    if (acc == 0x9e3779b9u) out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename F>
int timed(F launch, float *ms)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
    launch();  // warm-up
    hipError_t e = hipEventRecord(a, nullptr);
    launch();
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return (e == hipSuccess && hipGetLastError() == hipSuccess) ? 0 : -1;
}

}  // namespace

extern "C" {

// Kinds: 0 v_add_u32, 1 v_add3_u32, 2 v_pk_add_u16, 3 v_lshl_or_b32,
// 4 v_fma_f64, 5 v_cvt_f64_i32, 6 v_max3_i32, 7 v_mad_u64_u32, 8 v_add_f64,
// 9 v_max_f64, 10 v_cvt_f32_i32, 11 v_mul_lo_u32, 12 v_cvt_f64_u32,
// 13 v_sub_u32.  Writes the launch's
// wave-instructions per second of the timed form.  `out` is a device buffer
// of >= blocks uint32.
int peaks_valu(int kind, int blocks, int iters, uint32_t *out, double *winst_per_s)
{
    float ms = 0.f;
    int rc = -1;
    auto go = [&](auto k) {
        rc = timed([&] { hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, nullptr, out, 12345u, iters); }, &ms);
    };
    switch (kind) {
    case 0: go(valu_kernel<0>); break;
    case 1: go(valu_kernel<1>); break;
    case 2: go(valu_kernel<2>); break;
    case 3: go(valu_kernel<3>); break;
    case 4: go(valu_kernel<4>); break;
    case 5: go(valu_kernel<5>); break;
    case 6: go(valu_kernel<6>); break;
    case 7: go(valu_kernel<7>); break;
    case 8: go(valu_kernel<8>); break;
    case 9: go(valu_kernel<9>); break;
    case 10: go(valu_kernel<10>); break;
    case 11: go(valu_kernel<11>); break;
    case 12: go(valu_kernel<12>); break;
    case 13: go(valu_kernel<13>); break;
    default: return -1;
    }
    if (rc) return rc;
    *winst_per_s = (double)blocks * 4 /* waves */ * iters * CHAINS / (ms * 1e-3);
    return 0;
}

// LDS read bytes per second of one read form (see lds_kernel: 0 b32,
// 1 read2st64_b32, 2 b64, 3 read2st64_b64, 4 b128, 5 read2_b32 aligned,
// 6 read2_b32 straddling, 7 b64 and straddling read2_b32 alternating).  `out` is a device
// buffer of >= blocks * 256 uint32.
int peaks_lds(int form, int blocks, int iters, uint32_t *out, double *bytes_per_s)
{
    float ms = 0.f;
    int rc = -1;
    auto go = [&](auto k) {
        rc = timed([&] { hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, nullptr, out, iters); }, &ms);
    };
    switch (form) {
    case 0: go(lds_kernel<0>); break;
    case 1: go(lds_kernel<1>); break;
    case 2: go(lds_kernel<2>); break;
    case 3: go(lds_kernel<3>); break;
    case 4: go(lds_kernel<4>); break;
    case 5: go(lds_kernel<5>); break;
    case 6: go(lds_kernel<6>); break;
    case 7: go(lds_kernel<7>); break;
    default: return -1;
    }
    if (rc) return rc;
    // 64 bytes per lane per trip
    *bytes_per_s = (double)blocks * 256 * iters * 64.0 / (ms * 1e-3);
    return 0;
}

// Device copy of `bytes` (a multiple of 16) from src to dst: bytes read plus
// bytes written per second, and the time of one copy.
int peaks_copy(const void *src, void *dst, size_t bytes, int blocks, double *bytes_per_s, double *seconds)
{
    float ms = 0.f;
    const size_t n = bytes / 16;
    int rc = timed([&] {
        hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, nullptr, static_cast<const uint4 *>(src),
                           static_cast<uint4 *>(dst), n);
    }, &ms);
    if (rc) return rc;
    *seconds = ms * 1e-3;
    *bytes_per_s = 2.0 * (double)bytes / (ms * 1e-3);
    return 0;
}

}  // extern "C"
