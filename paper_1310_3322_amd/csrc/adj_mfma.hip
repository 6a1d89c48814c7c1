// Backward (adjoint) kernel on FP32 MFMA (gfx950): Baum-Welch E-step counts.
//
// The paper's learning mode runs the Baum-Welch function of its HMM stage
// (Sec. 2.7).  Its E-step is the scaled backward recursion; with the forward
// pass rescaled by exact powers of two (alphahat_t = alpha_t 2^-E_t,
// m_T = sum_i alphahat_T(i)) the scaled backward variables are
//   betahat_T = 1 / m_T,   w_{t+1} = B[:, o_{t+1}] o betahat_{t+1} 2^-e_{t+1},
//   betahat_t = A w_{t+1},
// so that gamma_t = alphahat_t o betahat_t sums to one and
// xi_t(i,j) = alphahat_t(i) A(i,j) w_{t+1}(j).  Each sequence s of weight w_s adds
//   n_pi += w_s gamma_1,  n_B[:, o_t] += w_s gamma_t,  C += w_s alphahat_t (x) w_{t+1}
// and n_A = A o C at the end: the gradient of sum_s w_s log P_s w.r.t. ln pi,
// ln A and ln B.
//
// Memory: the forward kernel stored alphahat every L = ceil(sqrt(Tmax)) steps
// (Tmax the longest sequence of the 16-sequence tile).  Walking the segments
// last to first, the wave recomputes alphahat for the L steps of a segment
// with the forward kernel's own step code (bit-identical), parks them in a
// per-wave buffer in global memory, and runs the backward recursion through
// the segment.  Memory per sequence grows with sqrt(T).
//
// Per step and tile of 16 sequences (layout as in the forward kernel):
//   betahat_t = A w_{t+1}            16x16x4 MFMAs, A fragments in registers
//   C += X^T W                       X = w_s alphahat_t, W = w_{t+1}: transposed
//                                    through a per-wave LDS tile so the 16
//                                    sequences become the MFMA contraction axis
//   n_B^T[o_t][i] += w_s gamma_t(i)  into the wave's LDS partial (slots that share
//                                    a symbol add in slot-rank rounds), written to
//                                    the tile's slab slot after each tile; or, when
//                                    the partial does not fit, to the global counts
//
// Global counts are 64-bit fixed-point sums (common.cuh) and each tile's sums are
// formed in an order fixed by its data, so the counts do not depend on which
// wave takes which tile.
#include <climits>

#include "common.cuh"
#include "fwd_step.cuh"
#include "kernels.h"

namespace hmm {
namespace {

constexpr int ADJ_CH = 16;                  // symbols per staging chunk in the recompute
constexpr int ADJ_SYM_STRIDE = ADJ_CH + 1;

template <int R>
struct AdjShape {
    static constexpr int NP = 16 * R;
    static constexpr int XS = NP + 4;       // padded row of the transposition tiles
    static constexpr int tile_floats = 2 * TILE * XS;               // X and W
    static constexpr int sym_ints = 2 * TILE * ADJ_SYM_STRIDE;
    static constexpr int per_wave_bytes = tile_floats * 4 + sym_ints * 4;
};

// Emission counts of a step into the LDS partial: the lane's 4 consecutive states
// of each 16-state block at (16 r + 4 g) ^ (4 o & swz) of symbol o's row, in rounds
// of the slot rank of the lane's symbol.
template <int R>
__device__ __forceinline__ void partial_add(float *nbl, int ot, int swz, int g, bool live, int rank,
                                            const float (&gm)[R][4]) {
    constexpr int NP = 16 * R;
    auto rmw = [&]() {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float *q = &nbl[ot * NP + ((16 * r + 4 * g) ^ (ot * 4 & swz))];
            float4 x = *(const float4 *)q;
            x.x += gm[r][0];
            x.y += gm[r][1];
            x.z += gm[r][2];
            x.w += gm[r][3];
            *(float4 *)q = x;
        }
    };
    if (live && rank == 0) rmw();
    for (int rr = 1; __ballot(live && rank >= rr) != 0; ++rr) {
        wave_lds_sync();
        if (live && rank == rr) rmw();
    }
}

__host__ __device__ inline int nb_swizzle_mask(int NP) { return (NP & (NP - 1)) == 0 ? NP - 4 : 0; }

template <int R, int WAVES, bool NBLDS>
__global__ void __launch_bounds__(WAVES * WAVE) k_adj_mfma(DevPtrs d, AdjLaunch a) {
    static_assert(!NBLDS || WAVES == 1, "the LDS partial holds one tile's counts");
    using SH = AdjShape<R>;
    constexpr int NP = SH::NP;
    constexpr int XS = SH::XS;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const int sl = lane & 15, g = lane >> 4;
    const int K = a.K, N = a.N, M = a.M;
    const int swz = nb_swizzle_mask(NP);
    const int F = fixed_exponent(*a.wmax, a.S, a.max_len);
    float *nbl = (float *)smem;                                        // [M][NP] when NBLDS
    uint32_t *ranktab = (uint32_t *)(smem + (NBLDS ? (size_t)M * NP * 4 : 0));  // [M] slot masks when NBLDS
    unsigned char *wbase = smem + (NBLDS ? (size_t)M * NP * 4 + (size_t)M * 4 : 0) + (size_t)wave * SH::per_wave_bytes;
    float *xt = (float *)wbase;                                        // [16][XS]
    float *wt = xt + TILE * XS;                                        // [16][XS]
    int32_t *sym = (int32_t *)(wt + TILE * XS);                        // [2][16][ADJ_SYM_STRIDE]

    const int slot = blockIdx.x * WAVES + wave;
    float *segf = a.seg + (size_t)slot * a.seg_stride;
    const int Lcap = (int)(a.seg_stride / (WAVE * (4 * R + 2)));
    float4 *seg_alpha = (float4 *)segf;                                // [Lcap][R][64]
    int32_t *seg_e = (int32_t *)(segf + (size_t)Lcap * WAVE * 4 * R);  // [Lcap][64]
    int32_t *seg_o = seg_e + (size_t)Lcap * WAVE;                      // [Lcap][64]

    const int G = gridDim.x;
    const int k_first = G >= K ? (int)(blockIdx.x % K) : (int)blockIdx.x;
    const int k_step = G >= K ? K : G;
    for (int k = k_first; k < K; k += k_step) {
        const int gbeg = a.gstart[k], gend = a.gstart[k + 1];
        const int ntiles = (gend - gbeg + TILE - 1) / TILE;
        const float *btk = a.bt + (size_t)k * M * NP;
        unsigned long long *B64k = a.B64 + (size_t)k * M * NP;  // [M][NP] symbol-major global counts
        if (NBLDS) {
            for (int i = lane; i < M * NP; i += WAVE) nbl[i] = 0.0f;
            for (int i = lane; i < M; i += WAVE) ranktab[i] = 0u;
            wave_lds_sync();
        }
        if (ntiles > 0) {
            const float *Ak = d.A + (size_t)k * N * N;
            float af[R][R][4], ab[R][R][4];
            load_fwd_fragments<R>(af, Ak, N, g, sl);
            load_bwd_fragments<R>(ab, Ak, N, g, sl);
            floatx4 C[R][R];  // per tile

            for (;;) {
                const int tile = wave_pop(&a.queue[k]);
                if (tile >= ntiles) break;

                const int pos = gbeg + tile * TILE + sl;
                const bool has = pos < gend;
                const int seq = has ? a.perm[pos] : 0;
                int32_t T = 0;
                int64_t off = 0;
                bool act = false;
                if (has) {
                    T = d.lengths[seq];
                    off = d.offsets[seq];
                    const int mk = d.model_of_seq[seq];
                    const bool bad = seq_bad(T, off, a.max_len, a.total) || mk < 0 || mk >= K;
                    if (bad) T = 0;
                    act = !bad && T > 0 && a.flag[pos] == 0;
                }
                // the checkpoint grid uses the forward kernel's tile maximum
                const int Tmax = wave_max_int(T);
                if (Tmax > 0) {
#pragma unroll
                for (int ri = 0; ri < R; ++ri)
#pragma unroll
                    for (int rj = 0; rj < R; ++rj) C[ri][rj] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                bool lane_nan = false;
                int L = 1;
                while (L * L < Tmax) ++L;
                if (!dbg_in(L - 1, Lcap, HMM_DEBUG_SEGMENT)) return;  // segment buffer too short (debug build)
                const int nseg = (Tmax + L - 1) / L;
                const float wgt = act ? (a.weight ? a.weight[seq] : 1.0f) : 0.0f;
                const int st_slot = lane >> 2, st_part = lane & 3;
                const int32_t st_T = __shfl(T, st_slot, WAVE);
                const int64_t st_off = __shfl(off, st_slot, WAVE);
                const int32_t *st_src = d.symbols + st_off;
                auto stage = [&](int buf, int t0) {
                    int32_t *dst = sym + buf * TILE * ADJ_SYM_STRIDE + st_slot * ADJ_SYM_STRIDE + st_part * (ADJ_CH / 4);
#pragma unroll
                    for (int u = 0; u < ADJ_CH / 4; ++u) {
                        const int p = t0 + st_part * (ADJ_CH / 4) + u;
                        int o = p < st_T ? st_src[p] : 0;
                        dst[u] = ((unsigned)o < (unsigned)M) ? o : 0;
                    }
                };

                float wn[R][4];      // w_{t+1}
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int v = 0; v < 4; ++v) wn[r][v] = 0.0f;

                for (int j = nseg - 1; j >= 0; --j) {
                    const int t0 = j * L;
                    const int t1 = min(t0 + L, Tmax);
                    // ---- recompute alphahat over [t0, t1) from checkpoint j
                    float acur[R][4];
                    int e0 = 0;
                    if (t0 < T) {
                        const float *src = a.ckpt + ((size_t)pos * a.nck + j) * NP;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            float4 q = *(const float4 *)&src[16 * r + 4 * g];
                            acur[r][0] = q.x;
                            acur[r][1] = q.y;
                            acur[r][2] = q.z;
                            acur[r][3] = q.w;
                        }
                        e0 = a.ckexp[(size_t)pos * a.nck + j];
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acur[r][v] = 0.0f;
                    }
                    stage(0, t0);
                    stage(1, t0 + ADJ_CH);
                    wave_lds_sync();
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        seg_alpha[(size_t)(0 * R + r) * WAVE + lane] = float4{acur[r][0], acur[r][1], acur[r][2], acur[r][3]};
                    seg_e[lane] = e0;
                    seg_o[lane] = sym[sl * ADJ_SYM_STRIDE];
                    for (int t = t0 + 1; t < t1; ++t) {
                        const int tl = t - t0;
                        if ((tl % ADJ_CH) == 0 && tl > 0) {
                            // chunk tl / ADJ_CH is staged; refill the buffer of the one before
                            stage(((tl / ADJ_CH) + 1) & 1, t + ADJ_CH);
                            wave_lds_sync();
                        }
                        const int o = sym[((tl / ADJ_CH) & 1) * TILE * ADJ_SYM_STRIDE + sl * ADJ_SYM_STRIDE + (tl % ADJ_CH)];
                        float4 b[R];
                        gather_b<R>(&btk[(size_t)o * NP], g, b);
                        floatx4 u[R];
                        tile_matvec<R>(af, acur, u);
                        int e;
                        emit_and_rescale<R>(u, b, acur, e);
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            seg_alpha[(size_t)(tl * R + r) * WAVE + lane] =
                                float4{acur[r][0], acur[r][1], acur[r][2], acur[r][3]};
                        seg_e[(size_t)tl * WAVE + lane] = e;
                        seg_o[(size_t)tl * WAVE + lane] = o;
                    }
                    // ---- backward through the segment
                    for (int t = t1 - 1; t >= t0; --t) {
                        const int tl = t - t0;
                        float al[R][4];
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            float4 q = seg_alpha[(size_t)(tl * R + r) * WAVE + lane];
                            al[r][0] = q.x;
                            al[r][1] = q.y;
                            al[r][2] = q.z;
                            al[r][3] = q.w;
                        }
                        const int et = seg_e[(size_t)tl * WAVE + lane];
                        const int ot = seg_o[(size_t)tl * WAVE + lane];
                        float part = 0.0f;
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int v = 0; v < 4; ++v) part += al[r][v];
                        const float m = sum_row_groups(part);
                        const bool live = act && t < T;          // gamma_t exists
                        const bool trans = act && t + 1 < T;     // xi_t exists
                        float be[R][4];
                        if (t + 1 < Tmax) {
                            floatx4 u[R];
                            tile_matvec<R>(ab, wn, u);
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int v = 0; v < 4; ++v) be[r][v] = u[r][v];
                            // C += X^T W with X = w_s alphahat_t, W = w_{t+1}
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                float4 xv = trans ? float4{wgt * al[r][0], wgt * al[r][1], wgt * al[r][2], wgt * al[r][3]}
                                                  : float4{0.0f, 0.0f, 0.0f, 0.0f};
                                float4 wv = trans ? float4{wn[r][0], wn[r][1], wn[r][2], wn[r][3]}
                                                  : float4{0.0f, 0.0f, 0.0f, 0.0f};
                                *(float4 *)&xt[sl * XS + 16 * r + 4 * g] = xv;
                                *(float4 *)&wt[sl * XS + 16 * r + 4 * g] = wv;
                            }
                            wave_lds_sync();
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                float xa[R], wb[R];
#pragma unroll
                                for (int r = 0; r < R; ++r) {
                                    xa[r] = xt[(4 * q + g) * XS + 16 * r + sl];
                                    wb[r] = wt[(4 * q + g) * XS + 16 * r + sl];
                                }
#pragma unroll
                                for (int ri = 0; ri < R; ++ri)
#pragma unroll
                                    for (int rj = 0; rj < R; ++rj)
                                        C[ri][rj] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[ri], wb[rj], C[ri][rj], 0, 0, 0);
                            }
                            wave_lds_sync();
                        } else {
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int v = 0; v < 4; ++v) be[r][v] = 0.0f;
                        }
                        if (t == T - 1) {
                            const float inv = 1.0f / m;
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int v = 0; v < 4; ++v) be[r][v] = inv;
                        }
                        // gamma_t -> emission counts (and initial counts at t = 0)
                        {
                            float gm[R][4];
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int i = 16 * r + 4 * g + v;
                                    gm[r][v] = (live && i < N) ? wgt * al[r][v] * be[r][v] : 0.0f;
                                    lane_nan |= !__builtin_isfinite(gm[r][v]);
                                }
                            if (NBLDS) {
                                partial_add<R>(nbl, ot, swz, g, live, slot_rank(ranktab, ot, sl), gm);
                            } else if (live) {
#pragma unroll
                                for (int r = 0; r < R; ++r)
#pragma unroll
                                    for (int v = 0; v < 4; ++v) {
                                        const int i = 16 * r + 4 * g + v;
                                        const float x = __builtin_isfinite(gm[r][v]) ? gm[r][v] : 0.0f;
                                        if (i < N) atomicAdd(&B64k[(size_t)ot * NP + quad_t(i)], to_fixed(x, F));
                                    }
                            }
                            if (live && t == 0) {
#pragma unroll
                                for (int r = 0; r < R; ++r)
#pragma unroll
                                    for (int v = 0; v < 4; ++v) {
                                        const int i = 16 * r + 4 * g + v;
                                        if (i < N) add_fixed(&a.pi64[(size_t)k * N + i], gm[r][v], F, &a.nanflag[k]);
                                    }
                            }
                        }
                        // w_t = b_t o betahat_t 2^-e_t for the step before
                        float4 b[R];
                        gather_b<R>(&btk[(size_t)ot * NP], g, b);
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            wn[r][0] = ldexp_f(b[r].x * be[r][0], -et);
                            wn[r][1] = ldexp_f(b[r].y * be[r][1], -et);
                            wn[r][2] = ldexp_f(b[r].z * be[r][2], -et);
                            wn[r][3] = ldexp_f(b[r].w * be[r][3], -et);
                        }
                    }
                }
                // this tile's n_A = A o C (row base opaque: the flush's addresses are formed
                // here, not kept live across the tile loop)
                {
                    const int rb = opaque(k * N + 4 * g);
#pragma unroll
                    for (int ri = 0; ri < R; ++ri)
#pragma unroll
                        for (int rj = 0; rj < R; ++rj)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int i = 16 * ri + 4 * g + v, jj = 16 * rj + sl;
                                const size_t e = (size_t)(rb + 16 * ri + v) * N + jj;
                                if (i < N && jj < N) add_fixed(&a.A64[e], d.A[e] * C[ri][rj][v], F, &a.nanflag[k]);
                            }
                }
                if (lane_nan) atomicOr(&a.nanflag[k], 1);
                }  // Tmax > 0
                if (NBLDS) {
                    // the tile's emission partial into its slab slot (zeros for an empty tile)
                    wave_lds_sync();
                    const int64_t slot = slab_slot(gbeg, k, tile);
                    float *dst = a.slab + (size_t)(dbg_in(slot, slab_slots(a.S, a.K), HMM_DEBUG_SLAB) ? slot : 0) * M * NP;
                    for (int idx = lane; idx < M * NP; idx += WAVE) {
                        const int o = idx / NP, ic = idx % NP;
                        dst[(size_t)o * NP + (ic ^ (o * 4 & swz))] = nbl[idx];
                        nbl[idx] = 0.0f;
                    }
                    wave_lds_sync();
                }
            }
        }
    }
}

template <int R, int WAVES, bool NBLDS>
size_t adj_lds_bytes(int M) {
    return (NBLDS ? (size_t)M * 16 * R * 4 + (size_t)M * 4 : 0) + (size_t)WAVES * AdjShape<R>::per_wave_bytes;
}

template <int R, int WAVES, bool NBLDS>
int occupancy_grid(int M, int cu_count, int K, bool set_attr) {
    auto kern = k_adj_mfma<R, WAVES, NBLDS>;
    const size_t lds = adj_lds_bytes<R, WAVES, NBLDS>(M);
    if (set_attr && lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVES * WAVE, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int grid = cu_count * per_cu;
    if (K > 0 && grid >= K) grid = (grid / K) * K;
    return grid;
}

constexpr size_t LDS_LIMIT = 160 * 1024;

// Which variant a shape takes: a one-wave workgroup with the emission partial in
// LDS (when it fits and the slab of per-tile partials stays within
// SLAB_MAX_BYTES), else four waves adding to the global counts.
template <int R>
bool use_partial(int M, int S, int K) {
    if (slab_slots(S, K) * M * 16 * R * 4 > SLAB_MAX_BYTES) return false;
    return adj_lds_bytes<R, 1, true>(M) <= LDS_LIMIT;
}

template <int R>
int grid_for(int M, int S, int cu_count, int K, bool set_attr, int *waves) {
    if (use_partial<R>(M, S, K)) {
        *waves = 1;
        return occupancy_grid<R, 1, true>(M, cu_count, K, set_attr);
    }
    *waves = 4;
    return occupancy_grid<R, 4, false>(M, cu_count, K, set_attr);
}

template <int R>
hipError_t launch_r(const DevPtrs &d, const AdjLaunch &a, int cu_count, hipStream_t st) {
    int waves = 4;
    const int full = grid_for<R>(a.M, a.S, cu_count, a.K, true, &waves);
    const int grid = persistent_grid(full, tile_bound(a.S, a.K, false, TILE), waves, a.K, a.max_grid);
    if (grid * waves > a.seg_slots) return hipErrorInvalidValue;
    if (use_partial<R>(a.M, a.S, a.K)) {
        if (a.slab == nullptr) return hipErrorInvalidValue;
        k_adj_mfma<R, 1, true><<<grid, WAVE, adj_lds_bytes<R, 1, true>(a.M), st>>>(d, a);
    } else {
        if (a.B64 == nullptr) return hipErrorInvalidValue;
        k_adj_mfma<R, 4, false><<<grid, 4 * WAVE, adj_lds_bytes<R, 4, false>(a.M), st>>>(d, a);
    }
    return hipGetLastError();
}

}  // namespace

bool adj_mfma_supported(int NP) { return NP == 16 || NP == 32 || NP == 48 || NP == 64; }

bool adj_mfma_slab(int NP, int M, int S, int K) {
    switch (NP / 16) {
        case 1: return use_partial<1>(M, S, K);
        case 2: return use_partial<2>(M, S, K);
        case 3: return use_partial<3>(M, S, K);
        case 4: return use_partial<4>(M, S, K);
        default: return false;
    }
}

int adj_mfma_slots(int NP, int M, int S, int K, int cu_count) {
    int waves = 4, grid = 0;
    switch (NP / 16) {
        case 1: grid = grid_for<1>(M, S, cu_count, K, true, &waves); break;
        case 2: grid = grid_for<2>(M, S, cu_count, K, true, &waves); break;
        case 3: grid = grid_for<3>(M, S, cu_count, K, true, &waves); break;
        case 4: grid = grid_for<4>(M, S, cu_count, K, true, &waves); break;
        default: return 0;
    }
    return grid * waves;
}

int64_t adj_mfma_seg_stride(int NP, int max_len) {
    int L = 1;
    while ((int64_t)L * L < max_len) ++L;
    return (int64_t)L * WAVE * (4 * (NP / 16) + 2);
}

hipError_t launch_adj_mfma(const DevPtrs &d, const AdjLaunch &a, int cu_count, hipStream_t st) {
    switch (a.NP / 16) {
        case 1: return launch_r<1>(d, a, cu_count, st);
        case 2: return launch_r<2>(d, a, cu_count, st);
        case 3: return launch_r<3>(d, a, cu_count, st);
        case 4: return launch_r<4>(d, a, cu_count, st);
        default: return hipErrorInvalidValue;
    }
}

HMM_DEBUG_TAKE(debug_take_adj_mfma)

}  // namespace hmm
