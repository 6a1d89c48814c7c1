// Device helpers shared by the HIP kernels of libhmm_mi355x (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hmm.h"

namespace hmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr int TILE = 16;          // sequences per wave tile (the 16 columns of a 16x16 MFMA tile)
constexpr double LN2 = 0.693147180559945309417232121458176568;

// Host-visible launch parameters shared by the planner and the kernels.
struct Plan {
    int32_t K, N, M, NP, S;
    int32_t groups;        // 1 when every sequence is scored against every model, else K
    int32_t max_len;
    int64_t total_symbols;
    int32_t nbins;         // groups * (max_len + 1)
};

// Sum over the four 16-lane rows of a wave: lanes l, l^16, l^32, l^48 end
// with the same (bitwise identical) value.  v_permlane16_swap exchanges odd
// and even rows, v_permlane32_swap exchanges the two 32-lane halves; adding
// the pair is commutative, so every lane of a row group gets the same sum.
__device__ __forceinline__ float sum_row_groups(float x) {
    auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

__device__ __forceinline__ float wave_sum(float x) {
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, WAVE);
    return x;
}

__device__ __forceinline__ int wave_max_int(int x) {
    for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m, WAVE));
    return x;
}

// Orders LDS traffic between lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier that orders LDS traffic only.  __syncthreads also makes
// global memory coherent across the workgroup, which waits for every
// outstanding global load and store of the wave before the barrier; a step
// whose waves exchange data through LDS only would then lose the loads it
// issued one step ahead.  Here the fences name the local address space, so
// the barrier waits for LDS operations alone and global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Next item of a per-wave work queue: the old value of *head, the same in every
// lane, after adding 1.  Every lane takes part in the atomic (lane 0 adds 1, the
// others 0) and the result is read from the first lane, so the pop is not under
// a lane-dependent branch.  A pop written as `if (lane == 0) x = atomicAdd(..);
// x = readfirstlane(x)` may be merged by the compiler with a later branch on the
// same lane predicate (for example an output written by lane 0), rotating the
// loop so that the other lanes re-enter it without lane 0 and never leave.
// Call with every lane of the wave active.
__device__ __forceinline__ int wave_pop(int32_t *head) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int v = atomicAdd(head, lane == 0 ? 1 : 0);
    return __builtin_amdgcn_readfirstlane(v);
}

// Returns v unchanged but opaque to the optimiser, so that address arithmetic
// derived from it is not hoisted out of the enclosing loop (which would pin one
// register pair per unrolled load for the whole kernel).
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Exponent e with x = m * 2^e, m in [0.5, 1) (0 for x = 0, inf or NaN).
__device__ __forceinline__ int frexp_exp(float x) { return __builtin_amdgcn_frexp_expf(x); }
__device__ __forceinline__ float ldexp_f(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }

// ---- Order-independent count sums.  Expected counts are added as 64-bit
// fixed-point integers, v -> round(v 2^F): integer addition is associative, so
// a sum does not depend on the order in which waves and workgroups add to it,
// and the counts are the same from run to run.  Every count is bounded by
// sum_s |w_s| T_s <= S max_len max_s |w_s| (each step adds at most |w_s| to an
// entry: gamma and xi are probabilities), so with
//   F = 62 - ceil(log2 S) - ceil(log2 max_len) - e,  max_s |w_s| < 2^e,
// no sum reaches 2^62 and the resolution is 2^-62 of that bound.
__device__ __forceinline__ int ceil_log2_u(uint32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

__device__ __forceinline__ int fixed_exponent(uint32_t wmax_bits, int S, int max_len) {
    const float wmax = __uint_as_float(wmax_bits);
    if (!(wmax > 0.0f) || !(wmax <= 3.0e38f)) return 0;  // no weight to add, or none finite
    return 62 - ceil_log2_u((uint32_t)S) - ceil_log2_u((uint32_t)max(max_len, 1)) - frexp_exp(wmax);
}

// round(v 2^F) as a two's-complement 64-bit integer, for |v 2^F| < 2^62: the
// rounded magnitude x splits exactly into x = hi 2^32 + lo with hi = floor(x 2^-32)
// and 0 <= lo < 2^32 (lo keeps only bits of x, at most 24 of them, so it is a
// float without rounding); the sign is applied to the 64-bit result.
__device__ __forceinline__ unsigned long long to_fixed(float v, int F) {
    const float x = __builtin_rintf(ldexp_f(__builtin_fabsf(v), F));
    const float hf = __builtin_floorf(x * 2.3283064365386963e-10f);  // 2^-32
    const uint32_t lo = (uint32_t)__builtin_fmaf(hf, -4294967296.0f, x);
    const unsigned long long u = ((unsigned long long)(uint32_t)hf << 32) | lo;
    return v < 0.0f ? (unsigned long long)0 - u : u;
}

__device__ __forceinline__ float from_fixed(unsigned long long x, int F) {
    return (float)__builtin_ldexp((double)(long long)x, -F);
}

// Adds v to a fixed-point count; a non-finite v (from a non-finite weight) marks
// the model instead, whose counts then read NaN.
__device__ __forceinline__ void add_fixed(unsigned long long *dst, float v, int F, int32_t *nan_flag) {
    if (v == 0.0f) return;
    if (__builtin_isfinite(v))
        atomicAdd(dst, to_fixed(v, F));
    else
        atomicOr(nan_flag, 1);
}

// Slot order of repeated symbols in one step of a 16-sequence tile: each of the
// wave's lanes of slot `sl` sets bit sl in the entry of its symbol in `tab`
// (an LDS atomic OR, order-independent), reads the entry back and clears it;
// returns how many lower slots share the symbol (0 for the first occurrence).
// Adds to an LDS partial then go in rounds of equal rank, so the result does
// not depend on how the LDS serialises lanes that collide.
__device__ __forceinline__ int slot_rank(uint32_t *tab, int sym, int sl) {
    atomicOr(&tab[sym], 1u << sl);
    wave_lds_sync();
    const uint32_t m = tab[sym];
    wave_lds_sync();
    tab[sym] = 0u;
    return __popc(m & ((1u << sl) - 1u));
}

// The same for the waves of a cooperative tile, which all hold the tile's 16
// slots and advance step by step between workgroup barriers: one table for all
// of them, two 16-bit masks per word (symbols o and o ^ 1), two halves used by
// alternate steps.  Every wave sets the same bits, so a wave's own OR completes
// the mask it reads.  The entry of the previous step (other half, which no wave
// touches during this step) is cleared here; the caller clears the last step's
// entry after a tile's last step, before the barrier that ends the tile.
// tab: [2][m2] words, m2 = ceil(M / 2); parity = step index & 1.
__device__ __forceinline__ int slot_rank_shared(uint32_t *tab, int m2, int sym, int parity, int prev_sym,
                                                bool has_prev, int sl) {
    uint32_t *cur = tab + parity * m2;
    if (has_prev) tab[(parity ^ 1) * m2 + (prev_sym >> 1)] = 0u;
    const int sh = (sym & 1) << 4;
    atomicOr(&cur[sym >> 1], 1u << (sh + sl));
    wave_lds_sync();
    const uint32_t m = (cur[sym >> 1] >> sh) & 0xffffu;
    return __popc(m & ((1u << sl) - 1u));
}

// Sequence checks shared by all kernels: returns true when sequence s is
// malformed (length outside [0, max_len], range outside the symbol array).
__device__ __forceinline__ bool seq_bad(int32_t T, int64_t off, int32_t max_len, int64_t total) {
    return T < 0 || T > max_len || off < 0 || off + (int64_t)T > total;
}

// Bounds checks of the debug build (compiled with -DHMM_DEBUG): dbg_in(i, n,
// bit) is false when 0 <= i < n does not hold and then sets `bit` (one of the
// HMM_DEBUG_* bits of hmm.h) in the debug word of the translation unit; the
// caller keeps the access inside its buffer (or skips it).  hmm_debug_flags
// collects the words.  In a normal build the checks are constant true and
// vanish.
#ifdef HMM_DEBUG
namespace {
__device__ unsigned int g_debug_word;
}
__device__ __forceinline__ bool dbg_in(int64_t i, int64_t n, unsigned int bit) {
    const bool ok = i >= 0 && i < n;
    if (!ok) atomicOr(&g_debug_word, bit);
    return ok;
}
// Host side: returns the word of this translation unit and clears it.
#define HMM_DEBUG_TAKE(fn)                                                            \
    uint32_t fn() {                                                                 \
        unsigned int v = 0, z = 0;                                                  \
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_debug_word), sizeof(v)) != hipSuccess) \
            return 0x80000000u;                                                     \
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_debug_word), &z, sizeof(z)) != hipSuccess)  \
            return 0x80000000u;                                                     \
        return v;                                                                   \
    }
#else
__device__ __forceinline__ bool dbg_in(int64_t, int64_t, unsigned int) { return true; }
#define HMM_DEBUG_TAKE(fn) \
    uint32_t fn() { return 0; }
#endif

}  // namespace hmm
