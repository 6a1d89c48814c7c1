// Cooperative tile step for large state counts (NP = 16 R).
//
// One workgroup of R / BO waves advances one tile of 16 sequences of one
// model.  Wave w owns the BO 16-state output blocks r = BO w .. BO w + BO - 1:
// it keeps the MFMA A operand of A_k^T for those blocks (4 R BO registers per
// lane) and computes, for each owned block,
//   u[s][16 r + j] = sum_i alphahat[s][i] A_k[i][16 r + j]
// as 4 R chained 16x16x4 FP32 MFMAs whose B operand (all NP states of
// alphahat, loaded once for the BO chains) comes from the workgroup's
// exchange buffer in LDS.  Each step
// every wave writes its block of alpha~ = u o b and its block's share of the
// per-sequence sum; after one barrier every wave reads all blocks and all
// shares, forms c_t and its exponent e_t (identically in every wave, fixed
// summation order) while the next step's product runs on the unscaled alpha~,
// and scales the product by 2^-e_t.
//
// Lane layout inside a wave is the one of the 16x16x4 result tile: lane l
// holds sequence l % 16 and the four states 16 r + 4 (l / 16) + 0..3 of each
// owned block r.
#pragma once

#include "common.cuh"

namespace hmm {

template <int R>
struct CoopShape {
    static constexpr int NP = 16 * R;
    static constexpr int XROW = NP + 4;   // padded row of the exchange buffer (floats)
    // exchange buffer: [2][16][XROW] alpha~, then [2][R][16] block sums
    static constexpr int x_floats = 2 * TILE * XROW;
    static constexpr int p_floats = 2 * R * TILE;
    static constexpr int floats = x_floats + p_floats;
};

// A operand fragments of owned block r0 + b:
// af[b][rp][v] = A_k[16 rp + 4 g + v][16 (r0 + b) + sl].
template <int R, int BO>
__device__ __forceinline__ void coop_load_fwd_fragments(float (&af)[BO][R][4], const float *Ak, int N, int r0, int g,
                                                        int sl) {
    const int lane_off = opaque(4 * g * N + 16 * r0 + sl);
#pragma unroll
    for (int b = 0; b < BO; ++b)
#pragma unroll
        for (int rp = 0; rp < R; ++rp)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rp + 4 * g + v, j = 16 * (r0 + b) + sl;
                af[b][rp][v] = (i < N && j < N) ? Ak[lane_off + (16 * rp + v) * N + 16 * b] : 0.0f;
            }
}

// A operand fragments of A_k itself for beta = A w:
// ab[b][rp][v] = A_k[16 (r0 + b) + sl][16 rp + 4 g + v].
template <int R, int BO>
__device__ __forceinline__ void coop_load_bwd_fragments(float (&ab)[BO][R][4], const float *Ak, int N, int r0, int g,
                                                        int sl) {
    const int lane_off = opaque((16 * r0 + sl) * N + 4 * g);
#pragma unroll
    for (int b = 0; b < BO; ++b)
#pragma unroll
        for (int rp = 0; rp < R; ++rp)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * (r0 + b) + sl, j = 16 * rp + 4 * g + v;
                ab[b][rp][v] = (i < N && j < N) ? Ak[lane_off + 16 * b * N + 16 * rp + v] : 0.0f;
            }
}

// Per-sequence sum of the previous step from the block shares (fixed order).
template <int R>
__device__ __forceinline__ float coop_step_sum(const float *psum, int sl) {
    float cs = 0.0f;
#pragma unroll
    for (int w = 0; w < R; ++w) cs = cs + psum[w * TILE + sl];
    return cs;
}

// u[b] = (frag-matrix[b] . X) 2^-e over all NP states for each owned block b, X
// read from the exchange buffer rows (layout [16][XROW]).  Scaling the product
// rather than its operand gives the same values (a power of two commutes with
// FP32 rounding away from the subnormal range), takes 4 BO ldexps per lane
// instead of 4 R, and lets the chain start before e is known.  Each chain is a
// single accumulator in block order; the operands of block rp + 1 are loaded
// while the MFMAs of block rp issue, and scheduling barriers keep the compiler
// from hoisting every load.
// q0 is the lane's first float4 of the row (block rp = 0), which a caller may
// request before it forms e (the two LDS reads then overlap).
template <int R, int BO>
__device__ __forceinline__ void coop_matvec_q0(const float (&f)[BO][R][4], const float *xrow_base, float4 q0, int e,
                                               int g, int sl, floatx4 (&u)[BO]) {
#pragma unroll
    for (int b = 0; b < BO; ++b) u[b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const float *row = xrow_base + sl * CoopShape<R>::XROW + 4 * g;
    float4 qn = q0;
#pragma unroll
    for (int rp = 0; rp < R; ++rp) {
        const float4 q = qn;
        if (rp + 1 < R) qn = *(const float4 *)&row[16 * (rp + 1)];
        const float in[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < BO; ++b) u[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[b][rp][v], in[v], u[b], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int b = 0; b < BO; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) u[b][v] = ldexp_f(u[b][v], -e);
}

template <int R, int BO>
__device__ __forceinline__ void coop_matvec(const float (&f)[BO][R][4], const float *xrow_base, int e, int g, int sl,
                                            floatx4 (&u)[BO]) {
    const float4 q0 = *(const float4 *)&xrow_base[sl * CoopShape<R>::XROW + 4 * g];
    coop_matvec_q0<R, BO>(f, xrow_base, q0, e, g, sl, u);
}

// Fragments streamed from memory instead of registers, for state counts whose
// fragments and count accumulators do not fit the register file together.
// fr points at this lane's fragments of block rp = 0 of the wave, laid out
// [R rp][64 lanes][BO] float4 (v = 0..3 in the float4); the fragments of block
// rp + D are loaded while the MFMAs of block rp issue (each load's offset is
// opaque, so that its address is formed next to it rather than hoisted out of
// the step loop as one register pair per block).  Same chains and order as
// coop_matvec, so the results are bit-identical to it.
template <int R, int BO, int D>
__device__ __forceinline__ void coop_matvec_stream_q0(const float4 *fr, const float *xrow_base, float4 q0, int e, int g,
                                                      int sl, floatx4 (&u)[BO]) {
#pragma unroll
    for (int b = 0; b < BO; ++b) u[b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const float *row = xrow_base + sl * CoopShape<R>::XROW + 4 * g;
    float4 ring[D][BO];
#pragma unroll
    for (int dd = 0; dd < D; ++dd)
#pragma unroll
        for (int b = 0; b < BO; ++b) ring[dd][b] = fr[opaque(dd * WAVE * BO + b)];
    float4 qn = q0;
#pragma unroll
    for (int rp = 0; rp < R; ++rp) {
        const float4 q = qn;
        if (rp + 1 < R) qn = *(const float4 *)&row[16 * (rp + 1)];
        float4 f[BO];
#pragma unroll
        for (int b = 0; b < BO; ++b) f[b] = ring[rp % D][b];
        if (rp + D < R) {
#pragma unroll
            for (int b = 0; b < BO; ++b) ring[rp % D][b] = fr[opaque((rp + D) * WAVE * BO + b)];
        }
        const float in[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < BO; ++b) {
                const float a = v == 0 ? f[b].x : v == 1 ? f[b].y : v == 2 ? f[b].z : f[b].w;
                u[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, in[v], u[b], 0, 0, 0);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int b = 0; b < BO; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) u[b][v] = ldexp_f(u[b][v], -e);
}

template <int R, int BO, int D>
__device__ __forceinline__ void coop_matvec_stream(const float4 *fr, const float *xrow_base, int e, int g, int sl,
                                                   floatx4 (&u)[BO]) {
    const float4 q0 = *(const float4 *)&xrow_base[sl * CoopShape<R>::XROW + 4 * g];
    coop_matvec_stream_q0<R, BO, D>(fr, xrow_base, q0, e, g, sl, u);
}

// alpha~ block = u o b, its share of the per-sequence sum (identical in the 4
// lanes of a sequence).
__device__ __forceinline__ float coop_emit(const floatx4 &u, const float4 &b, float (&x)[4]) {
#pragma clang fp contract(off)
    x[0] = u[0] * b.x;
    x[1] = u[1] * b.y;
    x[2] = u[2] * b.z;
    x[3] = u[3] * b.w;
    const float part = ((x[0] + x[1]) + x[2]) + x[3];
    return sum_row_groups(part);
}

}  // namespace hmm
