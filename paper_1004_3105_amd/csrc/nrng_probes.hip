// nrng_probes.hip -- the issue-rate probe of single VALU instructions, used to
// weight the ALU roofline's operation counts by what each instruction costs
// to issue on this GPU.  Not part of the generation path.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

#include "nrng_launch.hpp"

namespace nrng {

// Issue-rate probe: 8 independent chains of one VALU instruction per lane
// (each instruction reads the result of the one 8 before it, so no chain
// waits on its own latency), xor-reduced into sink[g] for g < sink_len.
// Written as instructions so that exactly the named one repeats.
template <int OP>
__global__ __launch_bounds__(256) void probe_valu_kernel(uint32_t iters, uint32_t *sink, uint64_t sink_len)
{
    const uint64_t g = blockIdx.x * 256ull + threadIdx.x;
    uint32_t c = 0x9E3779B9u + blockIdx.x;
    uint64_t c64 = 0x9E3779B97F4A7C15ull + blockIdx.x;
    uint32_t a[8];
    uint64_t b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = threadIdx.x * 8u + j + 1u;
        b[j] = (uint64_t)a[j] << 20;
    }
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (OP == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(c));
            if constexpr (OP == 1) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[j]) : "v"(c));
            if constexpr (OP == 2) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[j]) : "v"(c));
            if constexpr (OP == 3) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(a[j]) : "v"(c));
            if constexpr (OP == 4) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(a[j]) : "v"(c));
            if constexpr (OP == 5) asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(a[j]));
            if constexpr (OP == 6) asm volatile("v_log_f32 %0, %0" : "+v"(a[j]));
            if constexpr (OP == 7) asm volatile("v_sin_f32 %0, %0" : "+v"(a[j]));
            if constexpr (OP == 8) asm volatile("v_sqrt_f32 %0, %0" : "+v"(a[j]));
            if constexpr (OP == 9) asm volatile("v_rcp_f32 %0, %0" : "+v"(a[j]));
            if constexpr (OP == 10) asm volatile("v_lshrrev_b64 %0, 30, %0" : "+v"(b[j]));
            if constexpr (OP == 11) asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(b[j]) : "v"(c64));
            if constexpr (OP == 12) asm volatile("v_mad_u64_u32 %0, vcc, %1, %1, %0" : "+v"(b[j]) : "v"(c) : "vcc");
            if constexpr (OP == 13) asm volatile("v_mad_i64_i32 %0, vcc, %1, %1, %0" : "+v"(b[j]) : "v"(c) : "vcc");
            if constexpr (OP == 14) asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(b[j]) : "v"(c64));
        }
    }
    uint64_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        r ^= (uint64_t)a[j] ^ b[j];
    if (g < sink_len)
        sink[g] = (uint32_t)(r ^ (r >> 32));
}

template <int... OPS>
static const void *probe_valu_fn(int op, std::integer_sequence<int, OPS...>)
{
    static const void *const tab[] = {(const void *)probe_valu_kernel<OPS>...};
    return op >= 0 && op < (int)sizeof...(OPS) ? tab[op] : nullptr;
}


int launch_probe_valu(int op, uint32_t iters, uint32_t *sink, uint64_t sink_len, uint32_t grid, hipStream_t s)
{
    const void *fn = probe_valu_fn(op, std::make_integer_sequence<int, kProbeValuOps>{});
    if (!fn)
        return (int)hipErrorInvalidValue;
    void *args[] = {&iters, &sink, &sink_len};
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, s);
}

}  // namespace nrng
