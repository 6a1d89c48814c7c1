// Plain per-sequence forward kernel (gfx950): the baseline the batched kernel
// is measured against, and the path for shapes the batched kernel does not take.
//
// One wave per (sequence, model) pair, in natural order, no sorting or
// batching.  Lane j holds the states j, j+64, ... ; the previous scaled
// forward vector sits in LDS and is read as a broadcast; A and B are read from
// global memory.  Textbook scaling (Sec. 2.7 "Forward"): c_t = sum_j
// alpha~_t(j), alphahat_t = alpha~_t / c_t, log P = sum_t ln c_t (accumulated
// in FP64).
#include <climits>

#include "common.cuh"
#include "kernels.h"

namespace hmm {
namespace {

constexpr int PLAIN_MAX_Q = (HMM_MAX_STATES + WAVE - 1) / WAVE;

__global__ void __launch_bounds__(64) k_fwd_plain(DevPtrs d, int K, int N, int M, int S, int all_pairs, int max_len,
                                                  int64_t total, float *out, int32_t *err) {
    __shared__ float alpha[HMM_MAX_STATES];
    const int lane = threadIdx.x;
    const int64_t p = blockIdx.x;
    const int s = all_pairs ? (int)(p / K) : (int)p;
    int k = all_pairs ? (int)(p % K) : d.model_of_seq[s];
    const int32_t T = d.lengths[s];
    const int64_t off = d.offsets[s];
    bool bad = seq_bad(T, off, max_len, total) || k < 0 || k >= K;
    if (bad) {
        if (lane == 0) {
            out[p] = NAN;
            atomicMin(err, s);
        }
        return;
    }
    const float *pi = d.pi + (size_t)k * N;
    const float *A = d.A + (size_t)k * N * N;
    const float *B = d.B + (size_t)k * N * M;
    const int32_t *o_seq = d.symbols + off;
    double ll = 0.0;
    bool dead = false, nan_sum = false;
    int sym_chunk = 0;
    for (int t = 0; t < T; ++t) {
        if ((t & (WAVE - 1)) == 0) sym_chunk = (t + lane < T) ? o_seq[t + lane] : 0;
        const int o = __shfl(sym_chunk, t & (WAVE - 1), WAVE);
        if (o < 0 || o >= M) {
            bad = true;
            break;
        }
        if (dead) continue;  // keep checking the remaining symbols
        float x[PLAIN_MAX_Q];
        float part = 0.0f;
#pragma unroll
        for (int q = 0; q < PLAIN_MAX_Q; ++q) {
            const int j = lane + WAVE * q;
            x[q] = 0.0f;
            if (j < N) {
                float u;
                if (t == 0) {
                    u = pi[j];
                } else {
                    u = 0.0f;
                    for (int i = 0; i < N; ++i) u += alpha[i] * A[(size_t)i * N + j];
                }
                x[q] = u * B[(size_t)j * M + o];
            }
            part += x[q];
        }
        const float c = wave_sum(part);
        if (!(c > 0.0f)) {
            dead = true;
            nan_sum = (c != 0.0f);
            continue;
        }
        ll += (double)logf(c);
        const float inv = 1.0f / c;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PLAIN_MAX_Q; ++q) {
            const int j = lane + WAVE * q;
            if (j < N) alpha[j] = x[q] * inv;
        }
        __syncthreads();
    }
    if (lane == 0) {
        float r = (bad || nan_sum) ? NAN : (dead ? -INFINITY : (float)ll);
        out[p] = r;
        if (bad) atomicMin(err, s);
    }
}

}  // namespace

hipError_t launch_fwd_plain(const DevPtrs &d, int K, int N, int M, int S, int all_pairs, int max_len, int64_t total,
                            float *ll, int32_t *err, hipStream_t st) {
    int64_t npairs = all_pairs ? (int64_t)S * K : (int64_t)S;
    if (npairs == 0) return hipSuccess;
    if (npairs > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fwd_plain, dim3((unsigned)npairs), dim3(64), 0, st, d, K, N, M, S, all_pairs, max_len, total,
                       ll, err);
    return hipGetLastError();
}

HMM_DEBUG_TAKE(debug_take_fwd_plain)

}  // namespace hmm
