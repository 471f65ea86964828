// Issue cost of the vector instructions the half-sweep kernels are made of,
// measured on the device this runs on: cycles per wave64 instruction per
// SIMD, with every SIMD holding 8 wavefronts and every wavefront running 16
// independent chains of one instruction (so neither latency nor dependence
// limits the rate).  Each instruction is written in inline assembly, so the
// loop holds exactly the instructions counted; all of it is register-only
// vector ALU work, and each thread stores one word of its chains at the end.
//
// Back-to-back v_mad_u64_u32 of one wavefront that write the same carry
// register get a one-cycle s_nop between them from the compiler; the other
// seven wavefronts of the SIMD issue meanwhile, so the figure is still the
// vector unit's rate.
//
// The rates do not add up in mixed code: an instruction that reads a scalar
// register is slow when such instructions follow each other, and nearly as
// fast as the all-vector forms when they alternate with them (the
// "alternating" cases), so a kernel's time is measured, not predicted, from
// these figures.
//
// Output: one line per instruction, then one JSON line with the same
// figures.  Cycles assume the nominal shader clock reported by the runtime;
// the ratios to v_add_u32 do not depend on the clock.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kIters = 2048;   // loop trips; 16 instructions per trip and wavefront
constexpr int kWavesPerSimd = 8;
constexpr int kBlock = 256;

#define VR_CHECK(x)                                                                         \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

#define VR_16(OP) OP(a0) OP(a1) OP(a2) OP(a3) OP(a4) OP(a5) OP(a6) OP(a7) \
                  OP(a8) OP(a9) OP(a10) OP(a11) OP(a12) OP(a13) OP(a14) OP(a15)

// One lane-mask / carry SGPR pair per chain (s_a0 .. s_a15), so consecutive
// instructions never write the same scalar register.
#define VR_SGPRS                                                                                      \
    uint64_t s_a0 = 0, s_a1 = 0, s_a2 = 0, s_a3 = 0, s_a4 = 0, s_a5 = 0, s_a6 = 0, s_a7 = 0, s_a8 = 0, \
             s_a9 = 0, s_a10 = 0, s_a11 = 0, s_a12 = 0, s_a13 = 0, s_a14 = 0, s_a15 = 0;
#define VR_SGPR_XOR                                                                                   \
    s_a0 ^ s_a1 ^ s_a2 ^ s_a3 ^ s_a4 ^ s_a5 ^ s_a6 ^ s_a7 ^ s_a8 ^ s_a9 ^ s_a10 ^ s_a11 ^ s_a12 ^ s_a13 ^ \
        s_a14 ^ s_a15

// 32-bit chains: a_i = OP(a_i, b, k)
#define VR_KERNEL32(NAME, ASM_OP)                                                                     \
    __global__ void __launch_bounds__(kBlock) NAME(uint32_t* out, uint32_t k, uint64_t mask) {        \
        const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;                                  \
        uint32_t a0 = tid, a1 = tid + 1, a2 = tid + 2, a3 = tid + 3, a4 = tid + 4, a5 = tid + 5,     \
                 a6 = tid + 6, a7 = tid + 7, a8 = tid + 8, a9 = tid + 9, a10 = tid + 10, a11 = tid + 11, \
                 a12 = tid + 12, a13 = tid + 13, a14 = tid + 14, a15 = tid + 15;                     \
        const uint32_t b = tid * 0x9E3779B9u;                                                        \
        const uint32_t vk = k ^ (tid & 1u); /* the constant, in a vector register */                 \
        const uint32_t v3 = 3u + (tid >> 31); /* a shift amount (3), in a vector register */         \
        VR_SGPRS                                                                                     \
        for (int it = 0; it < kIters; ++it) { VR_16(ASM_OP) }                                        \
        out[tid] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7 ^ a8 ^ a9 ^ a10 ^ a11 ^ a12 ^ a13 ^ a14 ^ a15 ^ \
                   (uint32_t)(VR_SGPR_XOR);                                                          \
    }

#define OP_ADD(a) asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(a) : "s"(k));
#define OP_ADD_V(a) asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(a) : "v"(b));
#define OP_ADD_C(a) asm volatile("v_add_u32_e32 %0, 7, %0" : "+v"(a));
#define OP_XOR3_V(a) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a) : "v"(b), "v"(vk));
#define OP_LSHR_S(a) asm volatile("v_lshrrev_b32_e32 %0, %1, %0" : "+v"(a) : "s"(k));
#define OP_ADD_L(a) asm volatile("v_add_u32_e32 %0, 0x9e3779b9, %0" : "+v"(a));
#define OP_SUB_V(a) asm volatile("v_sub_u32_e32 %0, %0, %1" : "+v"(a) : "v"(b));
#define OP_XOR_V(a) asm volatile("v_xor_b32_e32 %0, %1, %0" : "+v"(a) : "v"(b));
#define OP_XOR3_C(a) asm volatile("v_bitop3_b32 %0, %0, %1, 5 bitop3:0x96" : "+v"(a) : "v"(b));
#define OP_LSHLOR_V(a) asm volatile("v_lshl_or_b32 %0, %0, %1, %2" : "+v"(a) : "v"(v3), "v"(b));
#define OP_ALIGN_C(a) asm volatile("v_alignbit_b32 %0, %0, %1, 31" : "+v"(a) : "v"(b));
#define OP_ALIGN_V(a) asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(v3));
#define OP_CMP_V(a)                                                                     \
    {                                                                                   \
        asm volatile("v_cmp_gt_u32_e64 %0, %1, %2" : "=s"(s_##a) : "v"(vk), "v"(a));    \
        asm volatile("v_add_u32_e32 %0, 1, %0" : "+v"(a));                              \
    }
#define OP_XOR3(a) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a) : "v"(b), "s"(k));
#define OP_LSHLOR(a) asm volatile("v_lshl_or_b32 %0, %0, 3, %1" : "+v"(a) : "v"(b));
#define OP_LSHR(a) asm volatile("v_lshrrev_b32_e32 %0, 3, %0" : "+v"(a));
#define OP_CNDMASK(a) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a) : "v"(b), "s"(mask));
#define OP_MULHI(a) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a) : "s"(k));
#define OP_MULLO(a) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a) : "s"(k));
// compare into a lane mask (its own SGPR pair per chain, read at the end),
// then one add to move the chain on
#define OP_CMP(a)                                                                       \
    {                                                                                   \
        asm volatile("v_cmp_gt_u32_e64 %0, %1, %2" : "=s"(s_##a) : "s"(k), "v"(a));     \
        asm volatile("v_add_u32_e32 %0, 1, %0" : "+v"(a));                              \
    }

// Dependent variants: all 16 instructions of a trip on one chain.
#define VR_DEP16(OP) OP(a0) OP(a0) OP(a0) OP(a0) OP(a0) OP(a0) OP(a0) OP(a0) \
                     OP(a0) OP(a0) OP(a0) OP(a0) OP(a0) OP(a0) OP(a0) OP(a0)
#define OP_ADD_V_DEP(a) VR_DEP16(OP_ADD_V)
#define OP_XOR3_V_DEP(a) VR_DEP16(OP_XOR3_V)
#define OP_XOR3_S_DEP(a) VR_DEP16(OP_XOR3)
#define OP_ADD_V_PAIR(a) OP_ADD_V(a0) OP_ADD_V(a1) OP_ADD_V(a0) OP_ADD_V(a1) OP_ADD_V(a0) OP_ADD_V(a1) \
    OP_ADD_V(a0) OP_ADD_V(a1) OP_ADD_V(a0) OP_ADD_V(a1) OP_ADD_V(a0) OP_ADD_V(a1) OP_ADD_V(a0) OP_ADD_V(a1) \
    OP_ADD_V(a0) OP_ADD_V(a1)

VR_KERNEL32(k_add, OP_ADD)
VR_KERNEL32(k_add_v, OP_ADD_V)
VR_KERNEL32(k_add_c, OP_ADD_C)
VR_KERNEL32(k_xor3_v, OP_XOR3_V)
VR_KERNEL32(k_lshr_s, OP_LSHR_S)
VR_KERNEL32(k_add_l, OP_ADD_L)
VR_KERNEL32(k_sub_v, OP_SUB_V)
VR_KERNEL32(k_xor_v, OP_XOR_V)
VR_KERNEL32(k_xor3_c, OP_XOR3_C)
VR_KERNEL32(k_lshl_or_v, OP_LSHLOR_V)
VR_KERNEL32(k_align_c, OP_ALIGN_C)
VR_KERNEL32(k_align_v, OP_ALIGN_V)
VR_KERNEL32(k_cmp_v, OP_CMP_V)

// 32-bit kernels whose trip is one 16-instruction group given by ASM_GROUP.
#define VR_KERNEL32G(NAME, ASM_GROUP)                                                                 \
    __global__ void __launch_bounds__(kBlock) NAME(uint32_t* out, uint32_t k, uint64_t mask) {        \
        const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;                                  \
        uint32_t a0 = tid, a1 = tid + 1;                                                             \
        const uint32_t b = tid * 0x9E3779B9u;                                                        \
        const uint32_t vk = k ^ (tid & 1u);                                                          \
        (void)mask;                                                                                  \
        for (int it = 0; it < kIters; ++it) { ASM_GROUP(a0) }                                        \
        out[tid] = a0 ^ a1;                                                                          \
    }
VR_KERNEL32G(k_add_v_dep, OP_ADD_V_DEP)
VR_KERNEL32G(k_xor3_v_dep, OP_XOR3_V_DEP)
VR_KERNEL32G(k_xor3_s_dep, OP_XOR3_S_DEP)
VR_KERNEL32G(k_add_v_pair, OP_ADD_V_PAIR)

// Mixed: each trip alternates a fast-form instruction (all vector operands)
// with a slow-form one (a scalar operand), on 16 independent chains.
#define OP_MIX_XOR3(a) OP_XOR3_V(a) OP_ADD(a)
#define OP_MIX_MAD(a)                                                                                         \
    asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a) : "v"(b), "v"(vk));                    \
    asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a) : "s"(k));
VR_KERNEL32(k_mix_xor3_add, OP_MIX_XOR3)
VR_KERNEL32(k_mix_xor3_mulhi, OP_MIX_MAD)
VR_KERNEL32(k_xor3, OP_XOR3)
VR_KERNEL32(k_lshl_or, OP_LSHLOR)
VR_KERNEL32(k_lshr, OP_LSHR)
VR_KERNEL32(k_cndmask, OP_CNDMASK)
VR_KERNEL32(k_mul_hi, OP_MULHI)
VR_KERNEL32(k_mul_lo, OP_MULLO)
VR_KERNEL32(k_cmp_add, OP_CMP)

// 64-bit chains through the addend: a_i = b * k + a_i (v_mad_u64_u32), or a
// 64-bit shift.
#define VR_KERNEL64(NAME, ASM_OP)                                                                     \
    __global__ void __launch_bounds__(kBlock) NAME(uint32_t* out, uint32_t k, uint64_t mask) {        \
        const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;                                  \
        uint64_t a0 = tid + mask, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,   \
                 a6 = a0 + 6, a7 = a0 + 7, a8 = a0 + 8, a9 = a0 + 9, a10 = a0 + 10, a11 = a0 + 11,   \
                 a12 = a0 + 12, a13 = a0 + 13, a14 = a0 + 14, a15 = a0 + 15;                         \
        const uint32_t b = tid * 0x9E3779B9u;                                                        \
        const uint32_t vk = k ^ (tid & 1u); /* the multiplier, in a vector register */               \
        const uint64_t vmask = mask ^ (tid & 1u); /* a 64-bit addend, in vector registers */         \
        VR_SGPRS                                                                                     \
        for (int it = 0; it < kIters; ++it) { VR_16(ASM_OP) }                                        \
        const uint64_t r = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7 ^ a8 ^ a9 ^ a10 ^ a11 ^ a12 ^ a13 ^ a14 ^ a15 ^ \
                           (VR_SGPR_XOR);                                                            \
        out[tid] = (uint32_t)r ^ (uint32_t)(r >> 32);                                                \
    }

#define OP_MAD64(a) asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(a), "=s"(s_##a) : "v"(b), "s"(k));
#define OP_MAD64_V(a) asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(a), "=s"(s_##a) : "v"(b), "v"(vk));
#define OP_SHL64(a) asm volatile("v_lshlrev_b64 %0, 3, %0" : "+v"(a));

#define OP_LSA_S(a) asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(a) : "s"(mask));
#define OP_LSA_V(a) asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(a) : "v"(vmask));

VR_KERNEL64(k_mad_u64, OP_MAD64)
VR_KERNEL64(k_mad_u64_v, OP_MAD64_V)
VR_KERNEL64(k_lshl_b64, OP_SHL64)
VR_KERNEL64(k_lsa_s, OP_LSA_S)
VR_KERNEL64(k_lsa_v, OP_LSA_V)

// The acceptance code of one site appended to an accumulator, both ways the
// half-sweep can compute it (thresholds in scalar registers, the draw in a
// vector register): two compares into lane masks, two selects and a
// shift-or; or two 64-bit adds whose carries are the code bits, with the
// accumulator as the high word, and two shifts.  One chain step is one site.
__device__ __forceinline__ uint32_t vr_accept_cmp(uint32_t acc, uint32_t u, uint32_t t4, uint32_t t8) {
    uint32_t x;
    uint64_t m4, m8;
    asm volatile("v_cmp_gt_u32_e64 %[m4], %[t4], %[u]\n\t"
                 "v_cmp_gt_u32_e64 %[m8], %[t8], %[u]\n\t"
                 "s_nop 1\n\t"
                 "v_cndmask_b32_e64 %[x], 0, 1, %[m4]\n\t"
                 "v_cndmask_b32_e64 %[x], %[x], 2, %[m8]\n\t"
                 "v_lshl_or_b32 %[acc], %[acc], 3, %[x]"
                 : [acc] "+v"(acc), [x] "=&v"(x), [m4] "=&s"(m4), [m8] "=&s"(m8)
                 : [u] "v"(u), [t4] "s"(t4), [t8] "s"(t8));
    return acc;
}
template <int S>
__device__ __forceinline__ uint32_t vr_shl(uint32_t x) {
    uint32_t r;
    asm volatile("v_lshlrev_b32 %0, %1, %2" : "=v"(r) : "i"(S), "v"(x));
    return r;
}
__device__ __forceinline__ uint64_t vr_add64(uint64_t x, uint64_t k) {
    uint64_t r;
    asm volatile("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(k));
    return r;
}
__device__ __forceinline__ uint32_t vr_accept_add64(uint32_t acc, uint32_t u, uint64_t k4, uint64_t k48) {
    const uint64_t p = vr_add64(((uint64_t)vr_shl<2>(acc) << 32) | u, k4);
    return (uint32_t)(vr_add64(((uint64_t)vr_shl<1>((uint32_t)(p >> 32)) << 32) | (uint32_t)p, k48) >> 32);
}
// compares into VCC and adds with carry-in: acc = ((4 acc + b4) << 1) + b8,
// with the two wait states a VALU read of a VALU-written VCC needs
__device__ __forceinline__ uint32_t vr_accept_vcc(uint32_t acc, uint32_t u, uint32_t t4, uint32_t t8) {
    asm volatile("v_lshlrev_b32_e32 %[acc], 1, %[acc]\n\t"
                 "v_cmp_gt_u32_e32 vcc, %[t4], %[u]\n\t"
                 "s_nop 1\n\t"
                 "v_addc_co_u32_e32 %[acc], vcc, %[acc], %[acc], vcc\n\t"
                 "v_cmp_gt_u32_e32 vcc, %[t8], %[u]\n\t"
                 "s_nop 1\n\t"
                 "v_addc_co_u32_e32 %[acc], vcc, %[acc], %[acc], vcc"
                 : [acc] "+v"(acc)
                 : [u] "v"(u), [t4] "s"(t4), [t8] "s"(t8)
                 : "vcc");
    return acc;
}
#define OP_ACC_CMP(a) a = vr_accept_cmp(a, b, k, k >> 1);
#define OP_ACC_VCC(a) a = vr_accept_vcc(a, b, k, k >> 1);
#define OP_CMP32(a)                                                                     \
    {                                                                                   \
        asm volatile("v_cmp_gt_u32_e32 vcc, %0, %1" : : "s"(k), "v"(a) : "vcc");       \
        asm volatile("v_add_u32_e32 %0, 1, %0" : "+v"(a));                              \
    }
#define OP_CNDMASK32(a) asm volatile("v_cndmask_b32_e32 %0, %0, %1, vcc" : "+v"(a) : "v"(b));
#define OP_CNDMASK_VCC64(a) asm volatile("v_cndmask_b32_e64 %0, %0, %1, vcc" : "+v"(a) : "v"(b));
#define OP_MIX_CNDMASK32(a) OP_CNDMASK32(a) OP_ADD_V(a)
#define OP_ACC_ADD64(a) a = vr_accept_add64(a, b, mask, mask >> 1);
VR_KERNEL32(k_acc_cmp, OP_ACC_CMP)
VR_KERNEL32(k_acc_add64, OP_ACC_ADD64)
VR_KERNEL32(k_acc_vcc, OP_ACC_VCC)
VR_KERNEL32(k_cmp32_add, OP_CMP32)
VR_KERNEL32(k_cndmask32, OP_CNDMASK32)
VR_KERNEL32(k_cndmask_vcc64, OP_CNDMASK_VCC64)
VR_KERNEL32(k_mix_cndmask32_add, OP_MIX_CNDMASK32)

typedef void (*Kernel)(uint32_t*, uint32_t, uint64_t);

struct Case {
    const char* name;
    Kernel fn;
    int instr_per_op;  // vector instructions per chain step
    const char* per = "instruction";  // what one reported figure covers
};

}  // namespace

int main() {
    hipDeviceProp_t prop;
    VR_CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const double clock_hz = (double)prop.clockRate * 1e3;
    const int simds = cus * 4;
    const int grid = simds * kWavesPerSimd * 64 / kBlock;
    uint32_t* out = nullptr;
    VR_CHECK(hipMalloc(&out, sizeof(uint32_t) * (size_t)grid * kBlock));
    hipEvent_t t0, t1;
    VR_CHECK(hipEventCreate(&t0));
    VR_CHECK(hipEventCreate(&t1));
    // operands: s = one scalar register, v = vector registers only, c = an
    // inline constant
    const Case cases[] = {
        {"v_add_u32 (s)", k_add, 1},
        {"v_add_u32 (v)", k_add_v, 1},
        {"v_add_u32 (c)", k_add_c, 1},
        {"v_add_u32 (literal)", k_add_l, 1},
        {"v_add_u32 (v), one chain", k_add_v_dep, 1},
        {"v_add_u32 (v), two chains", k_add_v_pair, 1},
        {"v_sub_u32 (v)", k_sub_v, 1},
        {"v_xor_b32 (v)", k_xor_v, 1},
        {"v_bitop3_b32 (s)", k_xor3, 1},
        {"v_bitop3_b32 (v)", k_xor3_v, 1},
        {"v_bitop3_b32 (c)", k_xor3_c, 1},
        {"v_bitop3_b32 (v), one chain", k_xor3_v_dep, 1},
        {"v_bitop3_b32 (s), one chain", k_xor3_s_dep, 1},
        {"v_bitop3_b32 (v) / v_add_u32 (s) alternating", k_mix_xor3_add, 2},
        {"v_bitop3_b32 (v) / v_mul_hi_u32 (s) alternating", k_mix_xor3_mulhi, 2},
        {"v_lshl_or_b32 (c, v)", k_lshl_or, 1},
        {"v_lshl_or_b32 (v)", k_lshl_or_v, 1},
        {"v_alignbit_b32 (c)", k_align_c, 1},
        {"v_alignbit_b32 (v)", k_align_v, 1},
        {"v_lshrrev_b32 (c)", k_lshr, 1},
        {"v_lshrrev_b32 (s)", k_lshr_s, 1},
        {"v_cndmask_b32_e64 (s mask)", k_cndmask, 1},
        {"v_cmp_gt_u32_e64 (s) + v_add_u32 (c)", k_cmp_add, 2},
        {"v_cmp_gt_u32_e64 (v) + v_add_u32 (c)", k_cmp_v, 2},
        {"v_mul_hi_u32 (s)", k_mul_hi, 1},
        {"v_mul_lo_u32 (s)", k_mul_lo, 1},
        {"v_mad_u64_u32 (s)", k_mad_u64, 1},
        {"v_mad_u64_u32 (v)", k_mad_u64_v, 1},
        {"v_lshlrev_b64 (c)", k_lshl_b64, 1},
        {"v_lshl_add_u64 (s)", k_lsa_s, 1},
        {"v_lshl_add_u64 (v)", k_lsa_v, 1},
        {"v_cmp_gt_u32_e32 (s, into VCC) + v_add_u32 (c)", k_cmp32_add, 2},
        {"v_cndmask_b32_e32 (VCC)", k_cndmask32, 1},
        {"v_cndmask_b32_e64 (VCC)", k_cndmask_vcc64, 1},
        {"v_cndmask_b32_e32 (VCC) / v_add_u32 (v) alternating", k_mix_cndmask32_add, 2},
        {"acceptance code per site: compares, selects, shift-or", k_acc_cmp, 1, "site"},
        {"acceptance code per site: compares into VCC, adds with carry", k_acc_vcc, 1, "site"},
        {"acceptance code per site: two 64-bit adds, two shifts", k_acc_add64, 1, "site"},
    };
    const int n_cases = (int)(sizeof cases / sizeof cases[0]);
    double cyc[64];
    std::printf("device %s (%s), %d CUs, nominal clock %.0f MHz, %d wavefronts per SIMD\n", prop.name,
                prop.gcnArchName, cus, clock_hz / 1e6, kWavesPerSimd);
    for (int c = 0; c < n_cases; ++c) {
        hipLaunchKernelGGL(cases[c].fn, dim3(grid), dim3(kBlock), 0, 0, out, 0x9E3779B9u, 0x5555555555555555ull);
        VR_CHECK(hipGetLastError());
        VR_CHECK(hipDeviceSynchronize());
        const int reps = 5;
        VR_CHECK(hipEventRecord(t0, 0));
        for (int r = 0; r < reps; ++r)
            hipLaunchKernelGGL(cases[c].fn, dim3(grid), dim3(kBlock), 0, 0, out, 0x9E3779B9u, 0x5555555555555555ull);
        VR_CHECK(hipGetLastError());
        VR_CHECK(hipEventRecord(t1, 0));
        VR_CHECK(hipEventSynchronize(t1));
        float ms = 0.f;
        VR_CHECK(hipEventElapsedTime(&ms, t0, t1));
        ms /= reps;
        const double instr_per_simd = (double)kWavesPerSimd * kIters * 16 * cases[c].instr_per_op;
        cyc[c] = ms * 1e-3 * clock_hz / instr_per_simd;
        std::printf("%-56s %8.3f ms  %5.2f cycles per wave64 %s\n", cases[c].name, ms, cyc[c], cases[c].per);
    }
    std::printf("{\"probe\": \"valu_rates\", \"arch\": \"%s\", \"cus\": %d, \"clock_mhz\": %.0f, \"cycles\": {", prop.gcnArchName,
                cus, clock_hz / 1e6);
    for (int c = 0; c < n_cases; ++c) std::printf("%s\"%s\": %.3f", c ? ", " : "", cases[c].name, cyc[c]);
    std::printf("}}\n");
    VR_CHECK(hipFree(out));
    return 0;
}
