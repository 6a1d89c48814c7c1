// One step of the batched forward recursion on 16x16x4 FP32 MFMA tiles.
//
// Shared by the forward kernel and by the segment recompute of the backward
// kernel, which must reproduce the forward pass bit for bit.  Contraction is
// off in the emission product so that the compiler cannot fuse multiplies and
// adds differently in the two kernels.
//
// Register layout (one wave, tile of 16 sequences, NP = 16 R padded states):
// lane l holds sequence slot l % 16 and, for every 16-state block r, the four
// states 16 r + 4 (l / 16) + v, v = 0..3.
#pragma once

#include "common.cuh"

namespace hmm {

// A-operand fragments of A_k^T: af[r][rp][v] = A_k[16 rp + 4 g + v][16 r + sl].
template <int R>
__device__ __forceinline__ void load_fwd_fragments(float (&af)[R][R][4], const float *Ak, int N, int g, int sl) {
    const int lane_off = opaque(4 * g * N + sl);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int rp = 0; rp < R; ++rp)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rp + 4 * g + v, j = 16 * r + sl;
                af[r][rp][v] = (i < N && j < N) ? Ak[lane_off + (16 * rp + v) * N + 16 * r] : 0.0f;
            }
}

// A-operand fragments of A_k itself: ab[r][rp][v] = A_k[16 r + sl][16 rp + 4 g + v]
// (for beta_t = A_k w_{t+1}).
template <int R>
__device__ __forceinline__ void load_bwd_fragments(float (&ab)[R][R][4], const float *Ak, int N, int g, int sl) {
    const int lane_off = opaque(sl * N + 4 * g);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int rp = 0; rp < R; ++rp)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * r + sl, j = 16 * rp + 4 * g + v;
                ab[r][rp][v] = (i < N && j < N) ? Ak[lane_off + 16 * r * N + 16 * rp + v] : 0.0f;
            }
}

// out[s][16 r + 4 g + v] = sum_i frag-matrix[.][i] * in[s][i] for the tile:
// with af this is (alphahat A)[s][j]; with ab it is (A w)[s][i].
template <int R>
__device__ __forceinline__ void tile_matvec(const float (&f)[R][R][4], const float (&in)[R][4], floatx4 (&acc)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int rp = 0; rp < R; ++rp)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int r = 0; r < R; ++r)
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[r][rp][v], in[rp][v], acc[r], 0, 0, 0);
}

// Emission product, per-step sum over the sequence's states, and exact
// power-of-two rescale.  x = u o b; cs = sum x (identical in the 4 lanes of a
// sequence); e = exponent of cs; out = x * 2^-e.  Returns cs, writes e.
template <int R>
__device__ __forceinline__ float emit_and_rescale(const floatx4 (&u)[R], const float4 (&b)[R], float (&out)[R][4],
                                                  int &e) {
#pragma clang fp contract(off)
    float x[R][4];
    float part = 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        x[r][0] = u[r][0] * b[r].x;
        x[r][1] = u[r][1] * b[r].y;
        x[r][2] = u[r][2] * b[r].z;
        x[r][3] = u[r][3] * b[r].w;
#pragma unroll
        for (int v = 0; v < 4; ++v) part = part + x[r][v];
    }
    const float cs = sum_row_groups(part);
    e = frexp_exp(cs);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[r][v] = ldexp_f(x[r][v], -e);
    return cs;
}

// First step: u = pi (pi fragment pf[r][v] = pi_k[16 r + 4 g + v]).
template <int R>
__device__ __forceinline__ void pi_as_u(const float *pik, int N, int g, floatx4 (&u)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * r + 4 * g + v;
            u[r][v] = i < N ? pik[i] : 0.0f;
        }
}

template <int R>
__device__ __forceinline__ void gather_b(const float *row, int g, float4 (&b)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) b[r] = *(const float4 *)&row[16 * r + 4 * g];
}

}  // namespace hmm
