// Viterbi decoding (gfx950): the most likely hidden state path of each
// sequence under its own model (paper Sec. 2.7, the "Viterbi" function of the
// HMM stage), in the log domain:
//   delta_1(i) = ln pi[i] + ln B[i][o_1]
//   delta_t(j) = max_i (delta_{t-1}(i) + ln A[i][j]) + ln B[j][o_t],   psi_t(j) = first i attaining it
//   score = max_j delta_T(j),  q_T = first j attaining it,  q_{t-1} = psi_t(q_t).
//
// The step is a max-plus product, which the matrix cores do not execute, so it
// runs on the vector ALUs.  A wave holds 64 / NP length-sorted sequences of one
// model; lane (slot, j) owns state j of its sequence and keeps the column
// ln A[:, j] in registers.  Per step every lane publishes delta_{t-1}(j) in
// LDS, reads the NP values of its sequence (four per read), forms the NP
// candidates in index order and keeps the first maximum (strict comparison),
// then adds ln B[j][o_t] from the log-emission table ln B^T [K][M][NP].  The
// back-pointer psi_t(j) is one byte in a [sum T][NP] array in HBM laid out
// like the symbols (sequence s owns rows offsets[s] .. offsets[s] + T - 1), so
// the traceback of a sequence walks one contiguous region.  Every RN steps the
// scores of a sequence are shifted by their maximum (a common shift changes no
// arg-max) and the shifts add up in FP64, which keeps the FP32 values small
// and the score accurate to a few ulps of its magnitude.
#include <climits>

#include "common.cuh"
#include "kernels.h"

namespace hmm {
namespace {

constexpr int VWAVES = 4;  // waves per workgroup
constexpr int RN = 16;     // steps between shifts

// (value, index) maximum over the NP lanes of a group, first index on ties.
template <int NP>
__device__ __forceinline__ void group_argmax(float &v, int &idx) {
#pragma unroll
    for (int m = 1; m < NP; m <<= 1) {
        const float ov = __shfl_xor(v, m, WAVE);
        const int oi = __shfl_xor(idx, m, WAVE);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
}

template <int NP>
__device__ __forceinline__ float group_max(float v) {
#pragma unroll
    for (int m = 1; m < NP; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, WAVE));
    return v;
}

template <int NP>
__global__ void __launch_bounds__(VWAVES * WAVE) k_viterbi(DevPtrs d, VitLaunch v) {
    constexpr int SPW = WAVE / NP;  // sequences per wave
    __shared__ __align__(16) float dl_all[VWAVES][2][WAVE];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int slot = lane / NP, j = lane % NP;
    const int K = v.K, N = v.N, M = v.M;

    const int G = gridDim.x;
    const int k_first = G >= K ? (int)(blockIdx.x % K) : (int)blockIdx.x;
    const int k_step = G >= K ? K : G;
    for (int k = k_first; k < K; k += k_step) {
        const int gbeg = v.gstart[k], gend = v.gstart[k + 1];
        const int nunits = (gend - gbeg + SPW - 1) / SPW;
        if (nunits == 0) continue;
        // column j of ln A_k (states beyond N are impossible)
        float la[NP];
        {
            const float *Ak = d.A + (size_t)k * N * N;
#pragma unroll
            for (int i = 0; i < NP; ++i) la[i] = (i < N && j < N) ? logf(Ak[(size_t)i * N + j]) : -INFINITY;
        }
        const float lpi = j < N ? logf(d.pi[(size_t)k * N + j]) : -INFINITY;
        const float *lbk = v.lnbt + (size_t)k * M * NP;

        for (;;) {
            const int unit = wave_pop(&v.queue[k]);
            if (unit >= nunits) break;

            const int pos = gbeg + unit * SPW + slot;
            const bool has = pos < gend;
            const int seq = has ? v.perm[pos] : 0;
            int32_t T = 0;
            int64_t off = 0;
            bool bad = false;
            if (has) {
                T = d.lengths[seq];
                off = d.offsets[seq];
                bad = seq_bad(T, off, v.max_len, v.total);
                const int mk = d.model_of_seq[seq];
                bad |= (mk < 0 || mk >= K);
                if (bad) T = 0;
            }
            const int Tmax = __builtin_amdgcn_readfirstlane(wave_max_int(T));
            const int32_t *sq = T > 0 ? d.symbols + off : d.symbols;
            uint8_t *bp = v.bp + (T > 0 ? off : 0) * NP + j;
            double shift = 0.0;
            float del = -INFINITY;
            bool symbad = false;
            float fin_v = -INFINITY;
            int fin_i = 0;
            double fin_shift = 0.0;
            for (int t = 0; t < Tmax; ++t) {
                const bool live = t < T;
                int o = live ? sq[t] : 0;
                symbad |= live && (o < 0 || o >= M);
                o = ((unsigned)o < (unsigned)M) ? o : 0;
                const float lb = lbk[(size_t)o * NP + j];
                if (t == 0) {
                    del = lpi + lb;
                } else {
                    float *buf = dl_all[wave][t & 1];
                    buf[lane] = del;
                    wave_lds_sync();
                    const float4 *row = (const float4 *)(buf + slot * NP);
                    float best = -INFINITY;
                    int arg = 0;
#pragma unroll
                    for (int i4 = 0; i4 < NP / 4; ++i4) {
                        const float4 q = row[i4];
                        const float c0 = q.x + la[4 * i4], c1 = q.y + la[4 * i4 + 1];
                        const float c2 = q.z + la[4 * i4 + 2], c3 = q.w + la[4 * i4 + 3];
                        if (c0 > best) { best = c0; arg = 4 * i4; }
                        if (c1 > best) { best = c1; arg = 4 * i4 + 1; }
                        if (c2 > best) { best = c2; arg = 4 * i4 + 2; }
                        if (c3 > best) { best = c3; arg = 4 * i4 + 3; }
                    }
                    del = best + lb;
                    if (live) bp[(size_t)t * NP] = (uint8_t)arg;
                }
                if (t == T - 1) {  // uniform within a sequence's lanes
                    fin_v = del;
                    fin_i = j;
                    fin_shift = shift;
                    group_argmax<NP>(fin_v, fin_i);
                }
                if (((t + 1) % RN) == 0) {
                    float m = group_max<NP>(del);
                    if (!(m > -INFINITY && m < INFINITY)) m = 0.0f;
                    del = del - m;
                    shift += (double)m;
                }
            }
            int sb = symbad ? 1 : 0;
#pragma unroll
            for (int m = 1; m < NP; m <<= 1) sb |= __shfl_xor(sb, m, WAVE);
            if (has && j == 0) {
                float sc;
                if (bad || sb) {
                    sc = NAN;
                    atomicMin(v.err, seq);
                } else if (T == 0) {
                    sc = 0.0f;
                } else {
                    sc = (float)(fin_shift + (double)fin_v);
                }
                v.score[seq] = sc;
                if (T > 0) v.path[off + T - 1] = (bad || sb) ? -1 : fin_i;
            }
        }
    }
}

// Traceback: follows the back-pointers from q_T (left in path by the decoding
// kernel) down to q_1, one wave per sequence, sequences taken in the planner's
// length-sorted order so that a round of waves has similar lengths; sequences
// with an invalid symbol or model get -1 everywhere (their range is written
// only when it is valid).  The back-pointer rows of 64 steps are copied to the
// wave's LDS buffer at once (lane l brings the row of step t_hi - l, NP bytes),
// with the next 64 rows in flight; the chase then reads one byte per step at a
// wave-uniform LDS address, and lane l keeps q_{t_hi - l - 1} for one coalesced
// store per chunk.
template <int NP>
__global__ void __launch_bounds__(VWAVES * WAVE) k_viterbi_trace_wave(DevPtrs d, VitLaunch v) {
    constexpr int DW = NP / 4;
    __shared__ uint32_t rowbuf[VWAVES][2][WAVE * DW];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int64_t pos = (int64_t)blockIdx.x * VWAVES + wave;
    if (pos >= v.S) return;
    const int s = v.perm[pos];
    const int32_t T = d.lengths[s];
    const int64_t off = d.offsets[s];
    if (seq_bad(T, off, v.max_len, v.total) || T == 0) return;
    int32_t *q = v.path + off;
    const float sc = v.score[s];
    if (sc != sc) {
        for (int32_t t = lane; t < T; t += WAVE) q[t] = -1;
        return;
    }
    const uint32_t *bp = (const uint32_t *)(v.bp + off * NP);
    uint32_t nxt[DW];
    auto load_rows = [&](int t_hi) {
        const int t = t_hi - lane;
#pragma unroll
        for (int u = 0; u < DW; ++u) nxt[u] = t >= 1 ? bp[(size_t)t * DW + u] : 0u;
    };
    auto store_rows = [&](int b) {
#pragma unroll
        for (int u = 0; u < DW; ++u) rowbuf[wave][b][lane * DW + u] = nxt[u];
    };
    int cur = __builtin_amdgcn_readfirstlane(q[T - 1]);
    int t_hi = T - 1;
    int buf = 0;
    load_rows(t_hi);
    store_rows(0);
    while (t_hi >= 1) {
        const int n = min(WAVE, t_hi);  // steps t_hi .. t_hi - n + 1 in this chunk
        if (t_hi - n >= 1) load_rows(t_hi - n);
        wave_lds_sync();
        const uint8_t *rb = (const uint8_t *)rowbuf[wave][buf];
        int mine = 0;  // q_{t_hi - lane - 1}, the state this lane decodes
        for (int l = 0; l < n; ++l) {
            cur = __builtin_amdgcn_readfirstlane((int)rb[l * NP + cur]);
            if (lane == l) mine = cur;
        }
        if (lane < n) q[t_hi - lane - 1] = mine;
        t_hi -= n;
        buf ^= 1;
        if (t_hi >= 1) store_rows(buf);
    }
}

template <int NP>
hipError_t launch_t(const DevPtrs &d, const VitLaunch &v, int cu_count, hipStream_t st) {
    auto kern = k_viterbi<NP>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, VWAVES * WAVE, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const int grid = persistent_grid(cu_count * per_cu, tile_bound(v.S, v.K, false, WAVE / NP), VWAVES, v.K, v.max_grid);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(VWAVES * WAVE), 0, st, d, v);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_viterbi_trace_wave<NP>, dim3((v.S + VWAVES - 1) / VWAVES), dim3(VWAVES * WAVE), 0, st, d, v);
    return hipGetLastError();
}

}  // namespace

bool viterbi_supported(int NP) { return NP == 16 || NP == 32 || NP == 64; }

hipError_t launch_viterbi(const DevPtrs &d, const VitLaunch &v, int cu_count, hipStream_t st) {
    if (v.S == 0) return hipSuccess;
    switch (v.NP) {
        case 16: return launch_t<16>(d, v, cu_count, st);
        case 32: return launch_t<32>(d, v, cu_count, st);
        case 64: return launch_t<64>(d, v, cu_count, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hmm
