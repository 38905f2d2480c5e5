// valu_rates.hip -- issue cost of the VALU instruction classes the walk uses,
// on gfx950.  Standalone measurement tool (not part of libsdd.so): every
// lane runs 8 independent chains of one instruction (pure ALU inline asm,
// no memory operands) and the shader clock is measured as s_memtime cycles
// over s_memrealtime ticks (100 MHz).  Reported: cycles per wave64
// instruction per SIMD.  The walk's roofline weights its per-step
// instruction mix with these costs.
//
//   valu_rates [waves_per_SIMD=8] [iterations=20000]
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#define CH 8
#define REP(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)
template <int OP>
__global__ __launch_bounds__(256) void mb(float* out, unsigned long long* clk, int iters, float kf, uint32_t ku)
{
    float a[CH], b[CH]; uint32_t u[CH]; uint64_t q[CH];
    for (int j = 0; j < CH; ++j) { a[j] = 0.3f + 1e-4f * (threadIdx.x + j); b[j] = a[j] * 0.5f; u[j] = threadIdx.x * 2654435761u + j; q[j] = u[j]; }
    const unsigned long long c0 = clock64(), w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
#define F(j) \
        if (OP == 0) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(kf), "v"(a[(j + 1) % CH])); \
        if (OP == 1) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(a[j]) : "v"(kf)); \
        if (OP == 2) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(u[j]) : "v"(ku)); \
        if (OP == 3) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(q[j]) : "v"(u[j]), "v"(ku) : "vcc"); \
        if (OP == 4) asm volatile("v_exp_f32 %0, %0" : "+v"(a[j])); \
        if (OP == 5) asm volatile("v_bitop3_b32 %0, %0, %1, %1 bitop3:0x96" : "+v"(u[j]) : "v"(ku)); \
        if (OP == 6) { asm volatile("v_exp_f32 %0, %0" : "+v"(a[j])); asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(b[j]) : "v"(kf)); } \
        if (OP == 7) { asm volatile("v_exp_f32 %0, %0" : "+v"(a[j])); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(b[j]) : "v"(kf)); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(b[j]) : "v"(kf)); } \
        if (OP == 8) { asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(q[j]) : "v"(u[j]), "v"(ku) : "vcc"); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(b[j]) : "v"(kf)); } \
        if (OP == 9) { asm volatile("v_xor_b32 %0, %0, %1" : "+v"(u[j]) : "v"(ku)); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(b[j]) : "v"(kf)); }
        REP(F)
#undef F
    }
    const unsigned long long c1 = clock64(), w1 = wall_clock64();
    float s = 0; for (int j = 0; j < CH; ++j) s += a[j] + b[j] + (float)u[j] + (float)q[j];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    out[gid] = s;
    if (threadIdx.x == 0) { clk[2 * blockIdx.x] = c1 - c0; clk[2 * blockIdx.x + 1] = w1 - w0; }
}
template <int OP> void run(const char* name, int nops, float* out, unsigned long long* clk, unsigned long long* hclk, int blocks, int iters) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return;
    hipLaunchKernelGGL(mb<OP>, dim3(blocks), dim3(256), 0, 0, out, clk, 10, 0.999f, 0x9E3779B9u);
    if (hipDeviceSynchronize() != hipSuccess) return;
    (void)hipEventRecord(e0);
    hipLaunchKernelGGL(mb<OP>, dim3(blocks), dim3(256), 0, 0, out, clk, iters, 0.999f, 0x9E3779B9u);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0; (void)hipEventElapsedTime(&ms, e0, e1);
    if (hipMemcpy(hclk, clk, 2 * blocks * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess) return;
    double cyc = 0, wall = 0;
    for (int b = 0; b < blocks; ++b) { cyc += hclk[2 * b]; wall += hclk[2 * b + 1]; }
    const double ghz = cyc / (wall / 100e6) / 1e9;  // s_memrealtime runs at 100 MHz
    const double wave_ops = (double)blocks * 4 * iters * CH * nops;  // 4 waves per block
    const double per_simd = wave_ops / 1024.0;
    printf("%-22s %8.3f ms  clock %.3f GHz  %5.2f cycles per wave64 op per SIMD\n", name, ms, ghz, (ms * 1e-3 * ghz * 1e9) / per_simd);
}
int main(int argc, char** argv) {
    int wps = argc > 1 ? atoi(argv[1]) : 8;
    int blocks = 256 * wps;
    int iters = argc > 2 ? atoi(argv[2]) : 20000;
    float* out; unsigned long long* clk;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return 1;
    if (hipMalloc(&clk, (size_t)blocks * 2 * sizeof(unsigned long long)) != hipSuccess) return 1;
    unsigned long long* h = (unsigned long long*)malloc(blocks * 2 * sizeof(unsigned long long));
    printf("waves/SIMD %d, iters %d\n", wps, iters);
    run<0>("fma_f32", 1, out, clk, h, blocks, iters);
    run<1>("mul_f32", 1, out, clk, h, blocks, iters);
    run<2>("xor_b32", 1, out, clk, h, blocks, iters);
    run<3>("mad_u64_u32", 1, out, clk, h, blocks, iters);
    run<4>("exp_f32", 1, out, clk, h, blocks, iters);
    run<5>("bitop3_b32", 1, out, clk, h, blocks, iters);
    run<6>("exp+fma (per pair)", 1, out, clk, h, blocks, iters);
    run<7>("exp+2mul (per trio)", 1, out, clk, h, blocks, iters);
    run<8>("mad_u64+mul (pair)", 1, out, clk, h, blocks, iters);
    run<9>("xor+mul (pair)", 1, out, clk, h, blocks, iters);
    (void)hipFree(out); (void)hipFree(clk); free(h);
    return 0;
}
