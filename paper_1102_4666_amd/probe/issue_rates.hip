// Stand-alone measurement program (not part of the library): the issue cost
// of the vector-ALU instruction forms the path kernels are built from, in
// shader-clock cycles per wave64 instruction on one SIMD.  Each kernel runs
// eight independent chains of one instruction form per lane at eight waves
// per SIMD, so that issue, not latency, sets its duration; the shader clock
// during the kernel is read in-kernel (s_memtime against s_memrealtime at
// 100 MHz), so that the result does not depend on the clock the part ran at.
//
// Build and run (gfx950):
//   hipcc -O3 -std=c++17 --offload-arch=gfx950 \
//       -Xclang -target-feature -Xclang -packed-fp32-ops \
//       paper_1102_4666_amd/probe/issue_rates.hip -o issue_rates && ./issue_rates
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <vector>

namespace {

constexpr int kChains = 8;
constexpr int kBlocks = 8192; // 32 waves per SIMD over the run
constexpr int kIters = 8192;

enum Form {
    kFmacV, kFmacS, kMulV, kXorV, kXorS, kAddV, kFma3V, kMulNeg, kBitop3V, kBitop3S,
    kMadU64, kMulHi, kCvt, kAlignbit, kCmpSel, kExp, kLog, kSqrt, kSin, kFmaF64,
    kXor8Exp4, kNumForms
};

const char *kNames[kNumForms] = {
    "v_fmac_f32, vector operands", "v_fmac_f32, one scalar operand", "v_mul_f32, vector operands",
    "v_xor_b32, vector operands", "v_xor_b32, one scalar operand", "v_add_u32, vector operands",
    "v_fma_f32 (VOP3), three vector operands", "v_mul_f32 (VOP3) with negated operand",
    "v_bitop3_b32, vector operands", "v_bitop3_b32, one scalar operand", "v_mad_u64_u32",
    "v_mul_hi_u32", "v_cvt_f32_u32", "v_alignbit_b32", "v_cmp + v_cndmask (2 instructions)",
    "v_exp_f32", "v_log_f32", "v_sqrt_f32", "v_sin_f32", "v_fmac_f64",
    "8 v_xor_b32 + 4 v_exp_f32 (12 instructions)"};
const double kInsts[kNumForms] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 1, 1, 1, 1, 1, 1.5};

template <int F>
__global__ __launch_bounds__(256) void chains(uint32_t *out, unsigned long long *clk, int iters,
                                              uint32_t s, float sg)
{
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const unsigned long long t0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    uint32_t a[kChains];
    float f[kChains];
    double d[kChains];
    uint64_t q[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = gid * 7 + c + 1;
        f[c] = 1.0f + (float)(gid + c) * 1e-7f;
        d[c] = f[c];
        q[c] = a[c];
    }
    // vector-register copies of uniform operands
    uint32_t wv = 0xD2511F53u, kv = s;
    float sv = sg;
    asm volatile("" : "+v"(wv), "+v"(kv), "+v"(sv));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const int n = (c + 1) % kChains;
            if constexpr (F == kFmacV) f[c] = fmaf(f[n], sv, f[c]);
            if constexpr (F == kFmacS) f[c] = fmaf(f[n], sg, f[c]);
            if constexpr (F == kMulV) f[c] = f[c] * f[n];
            if constexpr (F == kXorV) a[c] = a[c] ^ a[n];
            if constexpr (F == kXorS) a[c] = a[c] ^ (s + it);
            if constexpr (F == kAddV) a[c] = a[c] + a[n];
            if constexpr (F == kFma3V) f[c] = fmaf(f[c], f[n], sv);
            if constexpr (F == kMulNeg) f[c] = -(f[c] * f[n]);
            if constexpr (F == kBitop3V) a[c] = __builtin_amdgcn_bitop3_b32(a[c], a[n], kv, 0x96);
            if constexpr (F == kBitop3S) a[c] = __builtin_amdgcn_bitop3_b32(a[c], a[n], s, 0x96);
            if constexpr (F == kMadU64) q[c] = (uint64_t)(uint32_t)(q[c] >> 32) * wv + q[c];
            if constexpr (F == kMulHi) a[c] = __umulhi(a[c], wv);
            if constexpr (F == kCvt) a[c] = __float_as_uint((float)a[c]);
            if constexpr (F == kAlignbit) a[c] = __builtin_amdgcn_alignbit(kv, a[c], 9u);
            if constexpr (F == kCmpSel) a[c] = (a[c] == 3u) ? a[n] : a[c];
            if constexpr (F == kExp) f[c] = __builtin_amdgcn_exp2f(f[c]);
            if constexpr (F == kLog) f[c] = __builtin_amdgcn_logf(f[c]);
            if constexpr (F == kSqrt) f[c] = __builtin_amdgcn_sqrtf(f[c]);
            if constexpr (F == kSin) f[c] = __builtin_amdgcn_sinf(f[c]);
            if constexpr (F == kFmaF64) d[c] = fma(d[n], (double)sv, d[c]);
            if constexpr (F == kXor8Exp4) {
                a[c] = a[c] ^ a[n];
                if (c % 2 == 0) f[c] = __builtin_amdgcn_exp2f(f[c]);
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        r += a[c] + __float_as_uint(f[c]) + (uint32_t)__double_as_longlong(d[c]) + (uint32_t)q[c];
    out[gid] = r;
    const unsigned long long t1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = t1 - t0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

typedef void (*Kernel)(uint32_t *, unsigned long long *, int, uint32_t, float);

template <int... F>
void fill(Kernel *k, std::integer_sequence<int, F...>)
{
    ((k[F] = chains<F>), ...);
}

bool ok(hipError_t e, const char *what)
{
    if (e != hipSuccess) fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return e == hipSuccess;
}

} // namespace

int main()
{
    const int n = kBlocks * 256;
    uint32_t *out = nullptr;
    unsigned long long *clk = nullptr;
    if (!ok(hipMalloc(&out, n * sizeof(uint32_t)), "hipMalloc") ||
        !ok(hipMalloc(&clk, 2 * kBlocks * sizeof(unsigned long long)), "hipMalloc"))
        return 1;
    std::vector<unsigned long long> h(2 * kBlocks);
    hipEvent_t e0, e1;
    if (!ok(hipEventCreate(&e0), "event") || !ok(hipEventCreate(&e1), "event")) return 1;
    Kernel k[kNumForms];
    fill(k, std::make_integer_sequence<int, kNumForms>{});
    // wave-instruction slots per SIMD: waves / SIMDs x iterations x chains
    const double slots = (double)n / 64 / 1024 * kIters * kChains;
    printf("| Instruction form | Cycles per wave64 instruction | Shader clock (GHz) |\n|---|---|---|\n");
    for (int rep = 0; rep < 2; ++rep) {
        for (int f = 0; f < kNumForms; ++f) {
            if (!ok(hipEventRecord(e0), "record")) return 1;
            hipLaunchKernelGGL(k[f], dim3(kBlocks), dim3(256), 0, 0, out, clk, kIters, 3u, 0.999f);
            if (!ok(hipGetLastError(), "launch") || !ok(hipEventRecord(e1), "record") ||
                !ok(hipEventSynchronize(e1), "sync"))
                return 1;
            float ms = 0;
            if (!ok(hipEventElapsedTime(&ms, e0, e1), "elapsed") ||
                !ok(hipMemcpy(h.data(), clk, h.size() * sizeof(h[0]), hipMemcpyDeviceToHost), "copy"))
                return 1;
            double sc = 0, sr = 0;
            for (int b = 0; b < kBlocks; ++b) {
                sc += (double)h[2 * b];
                sr += (double)h[2 * b + 1];
            }
            const double ghz = sc / sr * 0.1;
            const double cyc = ms * 1e-3 * ghz * 1e9 / (slots * kInsts[f]);
            if (rep == 1) printf("| %s | %.2f | %.3f |\n", kNames[f], cyc, ghz);
        }
    }
    (void)hipFree(out);
    (void)hipFree(clk);
    return 0;
}
