// Cooperative-tile backward (adjoint) kernel (gfx950): Baum-Welch E-step counts
// for state counts that need several waves per tile (N = 64 .. 256).
//
// Same mathematics as adj_mfma.hip (paper Sec. 2.7 "BalmWelch" E-step; scaled
// beta recursion of the power-of-two-rescaled forward pass):
//   betahat_T = 1 / m_T,  w_{t+1} = B[:, o_{t+1}] o betahat_{t+1} 2^-e_{t+1},
//   betahat_t = A w_{t+1},  gamma_t = alphahat_t o betahat_t,
//   n_pi += w_s gamma_1,  n_B[:, o_t] += w_s gamma_t,  C += w_s alphahat_t (x) w_{t+1},
//   n_A = A o C.
// One workgroup of R / BO waves per tile of 16 length-sorted sequences of one
// model; wave w owns the BO 16-state blocks BO w .. BO w + BO - 1 (the
// partition of the gradient's forward, fwd_coop.hip).  When the forward stored
// every step's alphahat (FULL), the workgroup walks the tile back once over
// the stored rows.  With checkpoints, for each sqrt(T) segment, last to first,
// the workgroup recomputes alphahat from the checkpoint with the cooperative
// forward step (bit-identical to the checkpointing forward), keeps each lane's
// own states in a per-workgroup buffer in global memory, then walks the
// segment backwards.  Per step of a walk: one
// barrier; w_{t+1} of all NP states is exchanged through LDS; wave w forms
// betahat for its rows (4 R BO MFMAs), adds its rows of C += X^T W (4 R BO
// MFMAs, the 16 sequences as the contraction axis, X transposed through a
// per-wave LDS tile), scatters its rows of gamma into the emission counts, and
// writes its blocks of w_t.
//
// Register budget.  A lane holds its rows of C (4 R BO floats) for the whole
// tile.  Up to N = 128 (BO = 1) the MFMA fragments of A_k^T (recompute) and of
// A_k (beta) stay in registers too; above that the three sets (3 N^2 floats per
// tile) exceed the register file of a CU, so the fragments are streamed from a
// pre-arranged copy in the workspace ([K][2][waves][R][64][BO] float4; 2 NP^2
// floats per model, resident in the XCD's L2) a few blocks ahead of use.
// Emission counts go to an LDS partial [M][NP] when it fits (one 16-state block
// per wave), written after each tile to the tile's slot of a slab of per-tile
// partials; else, in a FULL walk of a call that ran its own forward, each live
// step's weighted gamma overwrites the row just read and k_grows_* sum the rows
// by (model, symbol) afterwards; else they go straight to the symbol-major
// global counts with atomics.  Every global count
// is a 64-bit fixed-point sum (common.cuh), and every sum inside a tile is formed
// in an order fixed by the tile's data (MFMA accumulation in step order; adds to
// the LDS partial in slot-rank rounds), so the counts do not depend on which
// workgroup takes which tile or when.
#include <climits>

#include "common.cuh"
#include "coop_step.cuh"
#include "kernels.h"

namespace hmm {
namespace {

constexpr int SSEG = 64;     // steps of symbols staged at a time (a whole segment up to T = 4096)
constexpr int PACH = 16;     // symbols per staging chunk of the pipelined kernel (its LDS is full)
constexpr int STREAM_D = 3;  // blocks of streamed fragments in flight

// Blocks per wave: as in the forward (one up to 8 blocks, two above).
constexpr int adj_bo(int R) { return R > 8 ? 2 : 1; }

template <int R, int BO>
struct AdjCoopShape {
    static constexpr int NP = 16 * R;
    static constexpr int NW = R / BO;                        // waves per workgroup
    static constexpr int XROW = CoopShape<R>::XROW;
    static constexpr int xch_floats = CoopShape<R>::floats;  // recompute exchange
    static constexpr int w_floats = 2 * TILE * XROW;         // w exchange, double-buffered
    static constexpr int at_floats = NW * BO * TILE * 17;    // per-wave transposition tiles
    static constexpr int small_bytes = (xch_floats + w_floats + at_floats) * 4 + SSEG * TILE * 4;
};

// LDS partial of the emission counts: state i of symbol o at o * NP + (i ^ (4 o & swz)),
// swz = P - 4 for P the largest power of two dividing NP.  Rows start on the same
// bank (NP is a multiple of 32), so without the XOR the 16 slots of a step would
// all add into the same banks; with it the rows of different symbols land on
// different ones.  The XOR keeps 4-state groups aligned (float4 adds) and every
// state within its row, and it permutes each row, so the waves, which own
// disjoint states, also own disjoint addresses.
__host__ __device__ inline int nb_swz(int NP) { return (NP & -NP) - 4; }

// The two fragment sets of a wave: resident in registers, or streamed.
template <int R, int BO, bool STREAM>
struct AdjFrags;

template <int R, int BO>
struct AdjFrags<R, BO, false> {
    float af[BO][R][4], ab[BO][R][4];
    __device__ __forceinline__ void load(const float *Ak, int N, int r0, int g, int sl, const float4 *, int) {
        coop_load_fwd_fragments<R, BO>(af, Ak, N, r0, g, sl);
        coop_load_bwd_fragments<R, BO>(ab, Ak, N, r0, g, sl);
    }
    __device__ __forceinline__ void fwd(const float *x, float4 q0, int e, int g, int sl, floatx4 (&u)[BO]) const {
        coop_matvec_q0<R, BO>(af, x, q0, e, g, sl, u);
    }
    __device__ __forceinline__ void bwd(const float *x, int g, int sl, floatx4 (&u)[BO]) const {
        coop_matvec<R, BO>(ab, x, 0, g, sl, u);
    }
};

template <int R, int BO>
struct AdjFrags<R, BO, true> {
    const float4 *faf, *fab;
    // frag_k: model k's two sets; lane_w: offset of this wave's and lane's first float4
    __device__ __forceinline__ void load(const float *, int, int, int, int, const float4 *frag_k, int lane_w) {
        constexpr size_t set = (size_t)R * R * WAVE;  // float4 per set (NW waves x R blocks x 64 lanes x BO)
        faf = frag_k + lane_w;
        fab = frag_k + set + lane_w;
    }
    __device__ __forceinline__ void fwd(const float *x, float4 q0, int e, int g, int sl, floatx4 (&u)[BO]) const {
        coop_matvec_stream_q0<R, BO, STREAM_D>(faf, x, q0, e, g, sl, u);
    }
    __device__ __forceinline__ void bwd(const float *x, int g, int sl, floatx4 (&u)[BO]) const {
        coop_matvec_stream<R, BO, STREAM_D>(fab, x, 0, g, sl, u);
    }
};

template <int R, int BO, bool NBLDS, bool STREAM, bool FULL>
__global__ void __launch_bounds__(R / BO * WAVE) k_adj_coop(DevPtrs d, AdjLaunch a) {
    // the kernel of the other storage mode serves the call (a uniform exit before any barrier)
    if (FULL != grad_full(a.arow, a.rowpos, a.S, a.grad_rows)) return;
    using SH = AdjCoopShape<R, BO>;
    // emission counts into the LDS partial one step late, overlapped with the next step's MFMAs
    static_assert(!(NBLDS && STREAM), "the LDS partial serves one-block waves");
    constexpr bool DEFER = NBLDS;
    constexpr int NP = SH::NP;
    constexpr int NW = SH::NW;
    constexpr int XROW = SH::XROW;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ __align__(16) float xch[SH::xch_floats];
    __shared__ __align__(16) float wex[SH::w_floats];
    __shared__ float atile_all[SH::at_floats];
    __shared__ int32_t symseg[SSEG * TILE];
    __shared__ int32_t tile_sh;
    float *nbl = (float *)smem;  // [M][NP] emission-count partial when NBLDS
    // [2][ceil(M / 2)] words after the partial: slot masks of the symbols of a step
    uint32_t *ranktab = (uint32_t *)(smem + (size_t)a.M * NP * 4);
    const int m2 = (a.M + 1) / 2;

    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int r0 = BO * w;  // first owned 16-state block
    const int sl = lane & 15, g = lane >> 4;
    const int K = a.K, N = a.N, M = a.M;
    const int swz = nb_swz(NP);
    const int F = fixed_exponent(*a.wmax, a.S, a.max_len);
    float *xbuf = xch;
    float *psum = xch + CoopShape<R>::x_floats;
    float *atile = atile_all + w * BO * TILE * 17;  // [BO][16 s][17] own alphahat blocks, transposed reads

    // per-workgroup segment buffer: alphahat [Lcap][NW][BO][64] float4, then e and o [Lcap][NW][64]
    const int slot = blockIdx.x;
    float *segf = a.seg + (size_t)slot * a.seg_stride;
    const int Lcap = (int)(a.seg_stride / ((size_t)NW * WAVE * (4 * BO + 2)));
    float4 *seg_alpha = (float4 *)segf;
    int32_t *seg_e = (int32_t *)(segf + (size_t)Lcap * NW * WAVE * 4 * BO);
    int32_t *seg_o = seg_e + (size_t)Lcap * NW * WAVE;
    auto aidx = [&](int tl, int b) { return (((size_t)tl * NW + w) * BO + b) * WAVE + lane; };
    auto sidx = [&](int tl) { return ((size_t)tl * NW + w) * WAVE + lane; };

    int k_first, k_step;
    model_walk(K, (int)gridDim.x, (int)blockIdx.x, &k_first, &k_step);
    for (int k = k_first; k < K; k += k_step) {
        const int gbeg = a.gstart[k], gend = a.gstart[k + 1];
        const int ntiles = (gend - gbeg + TILE - 1) / TILE;
        const float *btk = a.bt + (size_t)k * M * NP;
        unsigned long long *B64k = a.B64 + (size_t)k * M * NP;  // [M][NP] symbol-major counts of model k
        if (NBLDS) {
            __syncthreads();
            for (int i = threadIdx.x; i < M * NP; i += blockDim.x) nbl[i] = 0.0f;
            for (int i = threadIdx.x; i < 2 * m2; i += blockDim.x) ranktab[i] = 0u;
            __syncthreads();
        }
        const float *Ak = d.A + (size_t)k * N * N;
        if (ntiles > 0) {
            AdjFrags<R, BO, STREAM> fr;
            fr.load(Ak, N, r0, g, sl, STREAM ? (const float4 *)a.frag + (size_t)k * 2 * R * R * WAVE : nullptr,
                    (w * R * WAVE + lane) * BO);
            floatx4 C[BO][R];  // rows 16 (r0 + b) + 4 g + v, columns 16 rj + sl; per tile

            for (;;) {
                if (threadIdx.x == 0) tile_sh = atomicAdd(&a.queue[k], 1);
                __syncthreads();
                const int tile = __builtin_amdgcn_readfirstlane(tile_sh);  // scalar exit: the loop holds barriers
                __syncthreads();
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
                const int Tmax = __builtin_amdgcn_readfirstlane(wave_max_int(T));
                if (Tmax > 0) {
#pragma unroll
                for (int b = 0; b < BO; ++b)
#pragma unroll
                    for (int rj = 0; rj < R; ++rj) C[b][rj] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                bool lane_nan = false;  // a non-finite count (from a non-finite weight) in this lane
                // checkpoints: segments of about sqrt(Tmax) steps, each recomputed
                // before it is walked; full storage: one walk over the stored rows
                int L = 1;
                if (FULL) {
                    L = Tmax;
                } else {
                    while (L * L < Tmax) ++L;
                    if (!dbg_in(L - 1, Lcap, HMM_DEBUG_SEGMENT)) return;  // segment buffer too short (debug build)
                }
                const int nseg = (Tmax + L - 1) / L;
                const float wgt = act ? (a.weight ? a.weight[seq] : 1.0f) : 0.0f;
                const int32_t *sbase = T > 0 ? d.symbols + off : d.symbols;
                const int tlim = T > 0 ? T - 1 : 0;
                float m_last = 1.0f;  // m_T of this lane's sequence (set in the last segment)
                int64_t rb = 0;       // first stored row of the sequence (full storage)
                if (FULL && T > 0) {
                    rb = a.rowpos[pos];
                    m_last = a.mlast[pos];
                }
                // alphahat, exponent and symbol of step t from the stored rows (steps past
                // the sequence's end read its last row; they are not used)
                auto fetch_full = [&](int t, float4 (&aq)[BO], int &et, int &ot) {
                    int64_t row = T > 0 ? rb + min(t, T - 1) : 0;
                    if (!dbg_in(row, a.grad_rows, HMM_DEBUG_GRAD_ROWS)) row = 0;
#pragma unroll
                    for (int b = 0; b < BO; ++b) aq[b] = *(const float4 *)&a.arow[(size_t)row * NP + 16 * (r0 + b) + 4 * g];
                    et = a.aexp[row];
                    const int o = sbase[min(t, tlim)];
                    ot = ((unsigned)o < (unsigned)M) ? o : 0;
                };
                // gamma_1 of this lane's states, added to n_pi after the tile (a global atomic
                // inside the step would make every step wait for all outstanding loads)
                float gpi[BO][4] = {};
                // Emission counts of the previous backward step, added to the LDS partial
                // during the next step.  A lane adds its 4 consecutive states of one symbol
                // with a plain 16-byte read-add-write (other waves own other state
                // blocks).  Slots of the tile that share a symbol at that step add in
                // rounds of their slot rank (the first occurrence in round 0, the second
                // in round 1, ...), so colliding lanes never add in the same instruction
                // and the sum is formed in slot order.
                float4 pend_gm[BO];
                int pend_ix[BO] = {};
                bool pend_on = false;
                int pend_rank = 0;
                int rank_prev = 0;      // symbol of the previous backward step (its mask entry is cleared next)
                bool rank_has_prev = false;
                auto rmw = [&]() {
#pragma unroll
                    for (int b = 0; b < BO; ++b) {
                        float4 q = *(const float4 *)&nbl[pend_ix[b]];
                        q.x += pend_gm[b].x;
                        q.y += pend_gm[b].y;
                        q.z += pend_gm[b].z;
                        q.w += pend_gm[b].w;
                        *(float4 *)&nbl[pend_ix[b]] = q;
                    }
                };
                auto flush_pending = [&]() {
                    if (pend_on && pend_rank == 0) rmw();
                    for (int r = 1; __ballot(pend_on && pend_rank >= r) != 0; ++r) {
                        wave_lds_sync();
                        if (pend_on && pend_rank == r) rmw();
                    }
                    pend_on = false;
                };
                // the w exchange buffer of "step Tmax" starts at zero
                for (int i = threadIdx.x; i < TILE * XROW; i += blockDim.x) wex[(Tmax & 1) * TILE * XROW + i] = 0.0f;

                for (int j = nseg - 1; j >= 0; --j) {
                    const int t0 = j * L;
                    const int t1 = min(t0 + L, Tmax);
                    // ---- symbols of the segment, SSEG steps at a time, staged by every
                    // wave (one load round trip per block; no staging registers live
                    // across the steps)
                    auto stage_syms = [&](int s0) {
                        for (int s = w * 4 + g; s < SSEG; s += NW * 4)
                            symseg[s * TILE + sl] = sbase[min(s0 + s, tlim)];
                    };
                    auto read_sym = [&](int t) {
                        const int o = symseg[((t - t0) % SSEG) * TILE + sl];
                        return ((unsigned)o < (unsigned)M) ? o : 0;
                    };
                    __syncthreads();
                    if constexpr (!FULL) {
                        stage_syms(t0);
                        // ---- recompute alphahat over [t0, t1) from checkpoint j
                        float x[BO][4];
#pragma unroll
                        for (int b = 0; b < BO; ++b) {
                            if (t0 < T) {
                                const float4 q =
                                    *(const float4 *)&a.ckpt[((size_t)pos * a.nck + j) * NP + 16 * (r0 + b) + 4 * g];
                                x[b][0] = q.x;
                                x[b][1] = q.y;
                                x[b][2] = q.z;
                                x[b][3] = q.w;
                            } else {
                                x[b][0] = x[b][1] = x[b][2] = x[b][3] = 0.0f;
                            }
                        }
                        int e_prev = (t0 < T) ? a.ckexp[(size_t)pos * a.nck + j] : 0;
#pragma unroll
                        for (int b = 0; b < BO; ++b) {
                            *(float4 *)&xbuf[(t0 & 1) * TILE * XROW + sl * XROW + 16 * (r0 + b) + 4 * g] =
                                float4{x[b][0], x[b][1], x[b][2], x[b][3]};
                            // block shares of sum_i alphahat_{t0}(i), in the forward's summation order
                            float part;
                            {
#pragma clang fp contract(off)
                                part = ((x[b][0] + x[b][1]) + x[b][2]) + x[b][3];
                            }
                            part = sum_row_groups(part);
                            if (g == 0) psum[(t0 & 1) * R * TILE + (r0 + b) * TILE + sl] = part;
                        }
                        __syncthreads();
#pragma unroll
                        for (int b = 0; b < BO; ++b) seg_alpha[aidx(0, b)] = float4{x[b][0], x[b][1], x[b][2], x[b][3]};
                        seg_e[sidx(0)] = e_prev;
                        seg_o[sidx(0)] = read_sym(t0);
                        if (t0 == T - 1) m_last = coop_step_sum<R>(psum + (t0 & 1) * R * TILE, sl);
                        for (int t = t0 + 1; t <= t1; ++t) {
                            // first operand of this step's product, requested with the block sums
                            const float *xprev = xbuf + ((t - 1) & 1) * TILE * XROW;
                            const float4 q0 = *(const float4 *)&xprev[sl * XROW + 4 * g];
                            int e = 0;
                            if (t > t0 + 1) {
                                // finish step t - 1: its sum and exponent, store alphahat_{t-1}
                                const float cs = coop_step_sum<R>(psum + ((t - 1) & 1) * R * TILE, sl);
                                e = frexp_exp(cs);
#pragma unroll
                                for (int b = 0; b < BO; ++b)
                                    seg_alpha[aidx(t - 1 - t0, b)] = float4{ldexp_f(x[b][0], -e), ldexp_f(x[b][1], -e),
                                                                            ldexp_f(x[b][2], -e), ldexp_f(x[b][3], -e)};
                                seg_e[sidx(t - 1 - t0)] = e;
                                if (t - 1 == T - 1) m_last = ldexp_f(cs, -e);
                            }
                            if (t == t1) break;
                            if (((t - t0) % SSEG) == 0) {  // segments longer than SSEG steps
                                __syncthreads();
                                stage_syms(t);
                                __syncthreads();
                            }
                            const int o = read_sym(t);
                            seg_o[sidx(t - t0)] = o;
                            // the emission row is requested before the matvec, which hides its latency
                            float4 bb[BO];
#pragma unroll
                            for (int b = 0; b < BO; ++b) bb[b] = *(const float4 *)&btk[(size_t)o * NP + 16 * (r0 + b) + 4 * g];
                            floatx4 u[BO];
                            // the checkpoint row enters unscaled (exponent 0), later rows by 2^-e
                            fr.fwd(xprev, q0, (t == t0 + 1) ? 0 : e, g, sl, u);
#pragma unroll
                            for (int b = 0; b < BO; ++b) {
                                const float part = coop_emit(u[b], bb[b], x[b]);
                                *(float4 *)&xbuf[(t & 1) * TILE * XROW + sl * XROW + 16 * (r0 + b) + 4 * g] =
                                    float4{x[b][0], x[b][1], x[b][2], x[b][3]};
                                if (g == 0) psum[(t & 1) * R * TILE + (r0 + b) * TILE + sl] = part;
                            }
                            lds_barrier();  // LDS exchange only; segment entries are the wave's own
                        }
                    }  // !FULL
                    // ---- backward through the segment; the segment entries of step t - 1
                    // are requested during step t, and the emission row of step t at its start
                    float4 aq_n[BO];
                    int et_n = 0, ot_n = 0;
                    if constexpr (FULL) {
                        fetch_full(t1 - 1, aq_n, et_n, ot_n);
                    } else {
#pragma unroll
                        for (int b = 0; b < BO; ++b) aq_n[b] = seg_alpha[aidx(t1 - 1 - t0, b)];
                        et_n = seg_e[sidx(t1 - 1 - t0)];
                        ot_n = seg_o[sidx(t1 - 1 - t0)];
                    }
                    for (int t = t1 - 1; t >= t0; --t) {
                        const int tl = t - t0;
                        float al[BO][4];
#pragma unroll
                        for (int b = 0; b < BO; ++b) {
                            al[b][0] = aq_n[b].x;
                            al[b][1] = aq_n[b].y;
                            al[b][2] = aq_n[b].z;
                            al[b][3] = aq_n[b].w;
                        }
                        const int et = et_n;
                        const int ot = ot_n;
                        float4 bb[BO];
#pragma unroll
                        for (int b = 0; b < BO; ++b) bb[b] = *(const float4 *)&btk[(size_t)ot * NP + 16 * (r0 + b) + 4 * g];
                        {
                            // unconditional (index clamped at the segment start), so that the
                            // wait for the emission row above can leave these loads in flight
                            const int tp = tl > 0 ? tl - 1 : 0;
                            if constexpr (FULL) {
                                fetch_full(t0 + tp, aq_n, et_n, ot_n);
                            } else {
#pragma unroll
                                for (int b = 0; b < BO; ++b) aq_n[b] = seg_alpha[aidx(tp, b)];
                                et_n = seg_e[sidx(tp)];
                                ot_n = seg_o[sidx(tp)];
                            }
                        }
                        const bool live = act && t < T;
                        const bool trans = act && t + 1 < T;
                        const float *wrow = wex + ((t + 1) & 1) * TILE * XROW;  // w_{t+1}, all states
                        float be[BO][4] = {};
                        const bool more = t + 1 < Tmax;
                        // The w row of step Tmax is zero, so the streamed variant runs the
                        // product there too (its result is unused: at t = Tmax - 1 beta is
                        // 1 / m_T or the sequence has ended); every path then issues the
                        // fragment loads, and the wait for the segment entries requested
                        // above can count them instead of waiting for every load.
                        if (STREAM || more) {
                            floatx4 u[BO];
                            fr.bwd(wrow, g, sl, u);
#pragma unroll
                            for (int b = 0; b < BO; ++b)
#pragma unroll
                                for (int v = 0; v < 4; ++v) be[b][v] = u[b][v];
                        }
                        if (t == T - 1) {
                            const float inv = 1.0f / m_last;
#pragma unroll
                            for (int b = 0; b < BO; ++b)
#pragma unroll
                                for (int v = 0; v < 4; ++v) be[b][v] = inv;
                        }
                        if (!DEFER && live) {
                            // emission counts before the C update, whose MFMAs cover the
                            // atomics' latency before the next step's first load is awaited.
                            // Global counts: one address per step, the lane's states at
                            // immediate offsets from it (per-state addresses were spilled
                            // to scratch, and each reload waited for every outstanding load)
                            // (the counts' quad-transposed layout puts the four lanes of a
                            // sequence on four adjacent words in each instruction)
                            const int ib = 16 * r0 + 4 * g;
                            if (FULL && a.srows != nullptr) {
                                // the weighted gamma of this step into its stored row (already read
                                // for this step), summed by symbol after the walk
                                float gmv[BO][4];
#pragma unroll
                                for (int b = 0; b < BO; ++b)
#pragma unroll
                                    for (int v = 0; v < 4; ++v) {
                                        const float gm = wgt * al[b][v] * be[b][v];
                                        lane_nan |= !__builtin_isfinite(gm);
                                        gmv[b][v] = gm;
                                        if (t == 0) gpi[b][v] = gm;
                                    }
                                int64_t row = rb + t;
                                if (!dbg_in(row, a.grad_rows, HMM_DEBUG_GRAD_ROWS)) row = 0;
#pragma unroll
                                for (int b = 0; b < BO; ++b)
                                    *(float4 *)&a.arow[(size_t)row * NP + 16 * (r0 + b) + 4 * g] =
                                        float4{gmv[b][0], gmv[b][1], gmv[b][2], gmv[b][3]};
                            } else {
                                unsigned long long *dst = B64k + (uint32_t)(ot * NP + 16 * r0 + g);
#pragma unroll
                                for (int b = 0; b < BO; ++b)
#pragma unroll
                                    for (int v = 0; v < 4; ++v) {
                                        const int i = ib + 16 * b + v;
                                        const float gm = wgt * al[b][v] * be[b][v];
                                        const bool fin = __builtin_isfinite(gm);
                                        lane_nan |= !fin;
                                        if (i < N) atomicAdd(dst + 16 * b + 4 * v, to_fixed(fin ? gm : 0.0f, F));
                                        if (t == 0) gpi[b][v] = gm;
                                    }
                            }
                        }
                        if (more) {
                            // C[own rows][all] += X^T W: X (own blocks) through the wave's tiles
#pragma unroll
                            for (int b = 0; b < BO; ++b)
#pragma unroll
                                for (int v = 0; v < 4; ++v)
                                    atile[(b * TILE + sl) * 17 + 4 * g + v] = trans ? wgt * al[b][v] : 0.0f;
                            wave_lds_sync();
                            if (DEFER) {
                                // all operands of the C update first; the deferred emission
                                // counts then run in the LDS while the MFMAs issue
                                float xa[4][BO], wb[4][R];
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
                                    const int s = 4 * q + g;
#pragma unroll
                                    for (int b = 0; b < BO; ++b) xa[q][b] = atile[(b * TILE + s) * 17 + sl];
#pragma unroll
                                    for (int rj = 0; rj < R; ++rj) wb[q][rj] = wrow[s * XROW + 16 * rj + sl];
                                }
                                flush_pending();
                                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                                for (int q = 0; q < 4; ++q)
#pragma unroll
                                    for (int rj = 0; rj < R; ++rj)
#pragma unroll
                                        for (int b = 0; b < BO; ++b)
                                            C[b][rj] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[q][b], wb[q][rj], C[b][rj],
                                                                                          0, 0, 0);
                            } else {
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
                                    const int s = 4 * q + g;
                                    float xa[BO];
#pragma unroll
                                    for (int b = 0; b < BO; ++b) xa[b] = atile[(b * TILE + s) * 17 + sl];
#pragma unroll
                                    for (int rj = 0; rj < R; ++rj) {
                                        const float wb = wrow[s * XROW + 16 * rj + sl];
#pragma unroll
                                        for (int b = 0; b < BO; ++b)
                                            C[b][rj] =
                                                __builtin_amdgcn_mfma_f32_16x16x4f32(xa[b], wb, C[b][rj], 0, 0, 0);
                                    }
                                    if (STREAM) __builtin_amdgcn_sched_barrier(0);
                                }
                            }
                            wave_lds_sync();
                        } else if (DEFER) {
                            flush_pending();
                        }
                        if (DEFER) {
                            // this step's emission counts wait in registers for the next step,
                            // with the slot rank of their symbol among the tile's slots
                            const int rank = slot_rank_shared(ranktab, m2, ot, t & 1, rank_prev, rank_has_prev, sl);
                            rank_prev = ot;
                            rank_has_prev = true;
#pragma unroll
                            for (int b = 0; b < BO; ++b) {
                                float gm[4];
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int i = 16 * (r0 + b) + 4 * g + v;
                                    gm[v] = (i < N) ? wgt * al[b][v] * be[b][v] : 0.0f;
                                    if (live && t == 0) gpi[b][v] = gm[v];
                                    lane_nan |= live && !__builtin_isfinite(gm[v]);
                                }
                                pend_gm[b] = float4{gm[0], gm[1], gm[2], gm[3]};
                                pend_ix[b] = ot * NP + ((16 * (r0 + b) + 4 * g) ^ (ot * 4 & swz));
                            }
                            pend_on = live;
                            pend_rank = rank;
                        }
                        // w_t = b_t o betahat_t 2^-e_t; zero where the sequence has ended or
                        // takes no part (its values may be inf / NaN and w enters the
                        // contraction over sequences of C)
#pragma unroll
                        for (int b = 0; b < BO; ++b) {
                            const float wn0 = live ? ldexp_f(bb[b].x * be[b][0], -et) : 0.0f;
                            const float wn1 = live ? ldexp_f(bb[b].y * be[b][1], -et) : 0.0f;
                            const float wn2 = live ? ldexp_f(bb[b].z * be[b][2], -et) : 0.0f;
                            const float wn3 = live ? ldexp_f(bb[b].w * be[b][3], -et) : 0.0f;
                            *(float4 *)&wex[(t & 1) * TILE * XROW + sl * XROW + 16 * (r0 + b) + 4 * g] =
                                float4{wn0, wn1, wn2, wn3};
                        }
                        lds_barrier();
                    }
                }
                if (DEFER) {
                    flush_pending();
                    if (rank_has_prev) ranktab[rank_prev >> 1] = 0u;  // the last step (t = 0) used half 0
                }
                // this tile's initial counts and n_A = A o C for this wave's rows; the row
                // base is opaque so that the flush's addresses are formed here and not kept
                // live across the tile loop
                {
                    const int rb = opaque(k * N + 16 * r0 + 4 * g);  // global row of (b, v) = rb + 16 b + v
                    const int ib = 16 * r0 + 4 * g;
#pragma unroll
                    for (int b = 0; b < BO; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (ib + 16 * b + v < N) add_fixed(&a.pi64[rb + 16 * b + v], gpi[b][v], F, &a.nanflag[k]);
#pragma unroll
                    for (int b = 0; b < BO; ++b)
#pragma unroll
                        for (int rj = 0; rj < R; ++rj)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int jj = 16 * rj + sl;
                                const size_t e = (size_t)(rb + 16 * b + v) * N + jj;
                                if (ib + 16 * b + v < N && jj < N)
                                    add_fixed(&a.A64[e], d.A[e] * C[b][rj][v], F, &a.nanflag[k]);
                            }
                }
                if (lane_nan) atomicOr(&a.nanflag[k], 1);
                }  // Tmax > 0
                if (NBLDS) {
                    // the tile's emission partial into its slab slot (zeros for an empty tile)
                    __syncthreads();
                    const int64_t slot = slab_slot(gbeg, k, tile);
                    float *dst = a.slab + (size_t)(dbg_in(slot, slab_slots(a.S, a.K), HMM_DEBUG_SLAB) ? slot : 0) * M * NP;
                    for (int idx = threadIdx.x; idx < M * NP; idx += blockDim.x) {
                        const int o = idx / NP, ic = idx % NP;
                        dst[(size_t)o * NP + (ic ^ (o * 4 & swz))] = nbl[idx];
                        nbl[idx] = 0.0f;
                    }
                }
            }
        }
    }
}

// Pipelined variant for 64 states with the LDS partial (one 16-state block
// per wave): 2 R waves per tile, in two groups that advance in lockstep,
// one barrier per step for all of them.  The backward group (waves 0 .. R-1)
// walks segment j backwards: betahat, the emission counts and w_t, as in
// k_adj_coop.  The recompute group (waves R .. 2R-1, wave R + w owning block w)
// meanwhile recomputes segment j - 1 from its checkpoint into the other half of
// the segment buffer.  For each backward step t of segment j both groups add
// to C += X^T W for their rows, the backward group the first R / 2 column
// blocks and the recompute group the others, from alphahat_t and w_{t+1} (the
// exchange row both read in that step), so that neither group's step carries
// all of it.  A tile thus takes nseg + 1 phases of at most L steps instead of
// 2 nseg, and the two groups' matrix-core chains share each SIMD.  Every
// quantity is formed by the same operations in the same order as in k_adj_coop.
template <int R>
__global__ void __launch_bounds__(2 * R * WAVE) k_adj_pipe(DevPtrs d, AdjLaunch a) {
    // full storage: the walk over the stored rows serves the call
    if (grad_full(a.arow, a.rowpos, a.S, a.grad_rows)) return;
    using SH = AdjCoopShape<R, 1>;
    constexpr int NP = SH::NP;
    constexpr int XROW = SH::XROW;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ __align__(16) float xch[SH::xch_floats];
    __shared__ __align__(16) float wex[SH::w_floats];
    __shared__ float atile_all[2 * SH::at_floats];  // one transposition tile per wave of both groups
    __shared__ int32_t sym[2][PACH * TILE];
    __shared__ float mlast[TILE];  // m_T of each sequence of the tile
    __shared__ int32_t tile_sh;
    float *nbl = (float *)smem;  // [M][NP] emission-count partial
    // [2][ceil(M / 2)] words after the partial: slot masks of the symbols of a step
    uint32_t *ranktab = (uint32_t *)(smem + (size_t)a.M * NP * 4);
    const int m2 = (a.M + 1) / 2;

    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const bool rec = wid >= R;          // recompute group (wave-uniform)
    const int w = rec ? wid - R : wid;  // owned 16-state block
    const int sl = lane & 15, g = lane >> 4;
    const int K = a.K, N = a.N, M = a.M;
    const int swz = nb_swz(NP);
    const int F = fixed_exponent(*a.wmax, a.S, a.max_len);
    float *xbuf = xch;
    float *psum = xch + CoopShape<R>::x_floats;
    float *atile = atile_all + wid * TILE * 17;  // [16 s][17] own alphahat block, transposed reads

    // segment buffer: two halves (segment parity), each alphahat [Lcap][R][64]
    // float4, then e and o [Lcap][R][64] int32
    float *segf = a.seg + (size_t)blockIdx.x * a.seg_stride;
    const int64_t half = a.seg_stride / 2;
    const int Lcap = (int)(half / ((int64_t)R * WAVE * 6));
    auto seg_alpha = [&](int j) { return (float4 *)(segf + (j & 1) * half); };
    auto seg_e = [&](int j) { return (int32_t *)(segf + (j & 1) * half + (int64_t)Lcap * R * WAVE * 4); };
    auto seg_o = [&](int j) { return (int32_t *)(segf + (j & 1) * half + (int64_t)Lcap * R * WAVE * 5); };
    auto sidx = [&](int tl) { return ((size_t)tl * R + w) * WAVE + lane; };

    int k_first, k_step;
    model_walk(K, (int)gridDim.x, (int)blockIdx.x, &k_first, &k_step);
    for (int k = k_first; k < K; k += k_step) {
        const int gbeg = a.gstart[k], gend = a.gstart[k + 1];
        const int ntiles = (gend - gbeg + TILE - 1) / TILE;
        const float *btk = a.bt + (size_t)k * M * NP;
        __syncthreads();
        for (int i = threadIdx.x; i < M * NP; i += blockDim.x) nbl[i] = 0.0f;
        for (int i = threadIdx.x; i < 2 * m2; i += blockDim.x) ranktab[i] = 0u;
        __syncthreads();
        const float *Ak = d.A + (size_t)k * N * N;
        if (ntiles > 0) {
            AdjFrags<R, 1, false> fr;
            fr.load(Ak, N, w, g, sl, nullptr, 0);
            // each group adds half of the transition counts: rows 16 w + 4 g + v,
            // columns 16 (rj0 + rj) + sl, rj0 = 0 (backward group) or R / 2; per tile
            constexpr int RH = R / 2;
            const int rj0 = rec ? RH : 0;
            floatx4 C[RH];
            // C[own rows][half] += X^T W for backward step t: alphahat_t of the own block,
            // weighted, through the wave's transposition tile; w_{t+1} from the exchange row
            auto c_update = [&](const float (&al)[4], bool trans, float wgt_, const float *wrow) {
#pragma unroll
                for (int v = 0; v < 4; ++v) atile[sl * 17 + 4 * g + v] = trans ? wgt_ * al[v] : 0.0f;
                wave_lds_sync();
                float xa[4], wb[4][RH];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int s = 4 * q + g;
                    xa[q] = atile[s * 17 + sl];
#pragma unroll
                    for (int rj = 0; rj < RH; ++rj) wb[q][rj] = wrow[s * XROW + 16 * (rj0 + rj) + sl];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int rj = 0; rj < RH; ++rj)
                        C[rj] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[q], wb[q][rj], C[rj], 0, 0, 0);
                wave_lds_sync();
            };

            for (;;) {
                if (threadIdx.x == 0) tile_sh = atomicAdd(&a.queue[k], 1);
                __syncthreads();
                const int tile = __builtin_amdgcn_readfirstlane(tile_sh);  // scalar exit: the loop holds barriers
                __syncthreads();
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
                const int Tmax = __builtin_amdgcn_readfirstlane(wave_max_int(T));
                if (Tmax > 0) {
#pragma unroll
                for (int rj = 0; rj < RH; ++rj) C[rj] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                bool lane_nan = false;  // a non-finite count (from a non-finite weight) in this lane
                int L = 1;
                while (L * L < Tmax) ++L;
                if (!dbg_in(L - 1, Lcap, HMM_DEBUG_SEGMENT)) return;  // segment buffer too short (debug build)
                const int nseg = (Tmax + L - 1) / L;
                const float wgt = act ? (a.weight ? a.weight[seq] : 1.0f) : 0.0f;
                const int32_t *sbase = T > 0 ? d.symbols + off : d.symbols;
                const int tlim = T > 0 ? T - 1 : 0;
                // backward group: gamma_1 (added after the tile) and the deferred emission
                // counts, added in slot-rank rounds as in k_adj_coop
                float gpi[4] = {};
                float4 pend_gm = {0.0f, 0.0f, 0.0f, 0.0f};
                int pend_ix = 0;
                bool pend_on = false;
                int pend_rank = 0;
                int rank_prev = 0;      // symbol of the previous backward step (its mask entry is cleared next)
                bool rank_has_prev = false;
                auto rmw = [&]() {
                    float4 q = *(const float4 *)&nbl[pend_ix];
                    q.x += pend_gm.x;
                    q.y += pend_gm.y;
                    q.z += pend_gm.z;
                    q.w += pend_gm.w;
                    *(float4 *)&nbl[pend_ix] = q;
                };
                auto flush_pending = [&]() {
                    if (pend_on && pend_rank == 0) rmw();
                    for (int r = 1; __ballot(pend_on && pend_rank >= r) != 0; ++r) {
                        wave_lds_sync();
                        if (pend_on && pend_rank == r) rmw();
                    }
                    pend_on = false;
                };
                for (int i = threadIdx.x; i < TILE * XROW; i += blockDim.x) wex[(Tmax & 1) * TILE * XROW + i] = 0.0f;
                if (threadIdx.x < TILE) mlast[threadIdx.x] = 1.0f;

                // recompute group state: symbols staged by its first wave, chunk c in sym[c & 1]
                int32_t nxt[PACH / 4];
                float x[4] = {};
                int e = 0, e_prev = 0;
                int t0B = 0;
                auto load_chunk = [&](int s0) {
#pragma unroll
                    for (int u = 0; u < PACH / 4; ++u) nxt[u] = sbase[min(s0 + 4 * u + g, tlim)];
                };
                auto store_chunk = [&](int c) {
#pragma unroll
                    for (int u = 0; u < PACH / 4; ++u) sym[c & 1][u * WAVE + lane] = nxt[u];
                };
                auto read_sym = [&](int t) {
                    const int tl = t - t0B, pp = tl % PACH;
                    int o = sym[(tl / PACH) & 1][(pp / 4) * WAVE + 16 * (pp % 4) + sl];
                    return ((unsigned)o < (unsigned)M) ? o : 0;
                };
                // entry 0 of a recomputed segment: the checkpoint itself
                auto store_entry0 = [&](int jB) {
                    seg_alpha(jB)[sidx(0)] = float4{x[0], x[1], x[2], x[3]};
                    seg_e(jB)[sidx(0)] = e_prev;
                    seg_o(jB)[sidx(0)] = read_sym(t0B);
                    if (t0B == T - 1 && w == 0 && g == 0) mlast[sl] = coop_step_sum<R>(psum + (t0B & 1) * R * TILE, sl);
                };
                // step tf's sum and exponent; alphahat_tf into the segment buffer
                auto finish = [&](int jB, int tf) {
                    const float cs = coop_step_sum<R>(psum + (tf & 1) * R * TILE, sl);
                    e = frexp_exp(cs);
                    seg_alpha(jB)[sidx(tf - t0B)] =
                        float4{ldexp_f(x[0], -e), ldexp_f(x[1], -e), ldexp_f(x[2], -e), ldexp_f(x[3], -e)};
                    seg_e(jB)[sidx(tf - t0B)] = e;
                    if (tf == T - 1 && w == 0 && g == 0) mlast[sl] = ldexp_f(cs, -e);
                };

                for (int p = 0; p <= nseg; ++p) {
                    const int jA = nseg - p;  // segment of the backward group (p >= 1)
                    const int jB = jA - 1;    // segment of the recompute group (>= 0)
                    const int t0A = jA * L;
                    const int LA = p >= 1 ? min(t0A + L, Tmax) - t0A : 0;
                    t0B = jB * L;
                    const int LB = jB >= 0 ? min(t0B + L, Tmax) - t0B : 0;
                    const int nint = max(LA, LB);
                    // the previous phase's segment entries and m_T values are visible after this
                    __syncthreads();
                    float4 aq_n = {0.0f, 0.0f, 0.0f, 0.0f};
                    int et_n = 0, ot_n = 0;
                    if (LA > 0) {
                        aq_n = seg_alpha(jA)[sidx(LA - 1)];
                        if (!rec) {
                            et_n = seg_e(jA)[sidx(LA - 1)];
                            ot_n = seg_o(jA)[sidx(LA - 1)];
                        }
                    }
                    for (int it = 0; it < nint; ++it) {
                        const int t = t0A + LA - 1 - it;  // backward step of both groups (it < LA)
                        if (!rec) {
                            if (it < LA) {
                                const int tl = t - t0A;
                                const float al[4] = {aq_n.x, aq_n.y, aq_n.z, aq_n.w};
                                const int et = et_n, ot = ot_n;
                                const float4 bb = *(const float4 *)&btk[(size_t)ot * NP + 16 * w + 4 * g];
                                {
                                    const int tp = tl > 0 ? tl - 1 : 0;
                                    aq_n = seg_alpha(jA)[sidx(tp)];
                                    et_n = seg_e(jA)[sidx(tp)];
                                    ot_n = seg_o(jA)[sidx(tp)];
                                }
                                const bool live = act && t < T;
                                float be[4] = {};
                                flush_pending();
                                if (t + 1 < Tmax) {
                                    floatx4 u[1];
                                    fr.bwd(wex + ((t + 1) & 1) * TILE * XROW, g, sl, u);
#pragma unroll
                                    for (int v = 0; v < 4; ++v) be[v] = u[0][v];
                                    c_update(al, act && t + 1 < T, wgt, wex + ((t + 1) & 1) * TILE * XROW);
                                }
                                if (t == T - 1) {
                                    const float inv = 1.0f / mlast[sl];
#pragma unroll
                                    for (int v = 0; v < 4; ++v) be[v] = inv;
                                }
                                // this step's emission counts wait in registers for the next step,
                                // with the slot rank of their symbol among the tile's slots
                                const int rank =
                                    slot_rank_shared(ranktab, m2, ot, t & 1, rank_prev, rank_has_prev, sl);
                                rank_prev = ot;
                                rank_has_prev = true;
                                float gm[4];
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int i = 16 * w + 4 * g + v;
                                    gm[v] = (i < N) ? wgt * al[v] * be[v] : 0.0f;
                                    if (live && t == 0) gpi[v] = gm[v];
                                    lane_nan |= live && !__builtin_isfinite(gm[v]);
                                }
                                pend_gm = float4{gm[0], gm[1], gm[2], gm[3]};
                                pend_ix = ot * NP + ((16 * w + 4 * g) ^ (ot * 4 & swz));
                                pend_on = live;
                                pend_rank = rank;
                                // w_t = b_t o betahat_t 2^-e_t; zero where the sequence has ended or takes no part
                                const float wn0 = live ? ldexp_f(bb.x * be[0], -et) : 0.0f;
                                const float wn1 = live ? ldexp_f(bb.y * be[1], -et) : 0.0f;
                                const float wn2 = live ? ldexp_f(bb.z * be[2], -et) : 0.0f;
                                const float wn3 = live ? ldexp_f(bb.w * be[3], -et) : 0.0f;
                                *(float4 *)&wex[(t & 1) * TILE * XROW + sl * XROW + 16 * w + 4 * g] =
                                    float4{wn0, wn1, wn2, wn3};
                            }
                        } else {
                            if (it < LB) {
                                if (it == 0) {
                                    // the segment's first symbols (read from the next step on, after the barrier)
                                    if (w == 0) {
                                        load_chunk(t0B);
                                        store_chunk(0);
                                        load_chunk(t0B + PACH);
                                        store_chunk(1);
                                        load_chunk(t0B + 2 * PACH);
                                    }
                                    // alphahat at the checkpoint of segment jB
                                    if (t0B < T) {
                                        const float4 q =
                                            *(const float4 *)&a.ckpt[((size_t)pos * a.nck + jB) * NP + 16 * w + 4 * g];
                                        x[0] = q.x;
                                        x[1] = q.y;
                                        x[2] = q.z;
                                        x[3] = q.w;
                                    } else {
                                        x[0] = x[1] = x[2] = x[3] = 0.0f;
                                    }
                                    e_prev = (t0B < T) ? a.ckexp[(size_t)pos * a.nck + jB] : 0;
                                    *(float4 *)&xbuf[(t0B & 1) * TILE * XROW + sl * XROW + 16 * w + 4 * g] =
                                        float4{x[0], x[1], x[2], x[3]};
                                    float part;
                                    {
#pragma clang fp contract(off)
                                        part = ((x[0] + x[1]) + x[2]) + x[3];
                                    }
                                    part = sum_row_groups(part);
                                    if (g == 0) psum[(t0B & 1) * R * TILE + w * TILE + sl] = part;
                                } else {
                                    const int tr = t0B + it;  // recomputed step
                                    // first operand of this step's product, requested with the block sums
                                    const float *xprev = xbuf + ((tr - 1) & 1) * TILE * XROW;
                                    const float4 q0 = *(const float4 *)&xprev[sl * XROW + 4 * g];
                                    if (it == 1)
                                        store_entry0(jB);
                                    else
                                        finish(jB, tr - 1);
                                    if (w == 0 && (it % PACH) == 0 && it >= PACH) {
                                        store_chunk(it / PACH + 1);
                                        load_chunk(tr + 2 * PACH);
                                    }
                                    const int o = read_sym(tr);
                                    seg_o(jB)[sidx(it)] = o;
                                    const float4 bb = *(const float4 *)&btk[(size_t)o * NP + 16 * w + 4 * g];
                                    floatx4 u[1];
                                    // the checkpoint row enters unscaled (exponent 0), later rows by 2^-e
                                    fr.fwd(xprev, q0, it == 1 ? 0 : e, g, sl, u);
                                    const float part = coop_emit(u[0], bb, x);
                                    *(float4 *)&xbuf[(tr & 1) * TILE * XROW + sl * XROW + 16 * w + 4 * g] =
                                        float4{x[0], x[1], x[2], x[3]};
                                    if (g == 0) psum[(tr & 1) * R * TILE + w * TILE + sl] = part;
                                }
                            }
                            if (it < LA && t + 1 < Tmax) {
                                const int tl = t - t0A;
                                const float al[4] = {aq_n.x, aq_n.y, aq_n.z, aq_n.w};
                                aq_n = seg_alpha(jA)[sidx(tl > 0 ? tl - 1 : 0)];
                                c_update(al, act && t + 1 < T, wgt, wex + ((t + 1) & 1) * TILE * XROW);
                            } else if (it < LA) {
                                const int tl = t - t0A;
                                aq_n = seg_alpha(jA)[sidx(tl > 0 ? tl - 1 : 0)];
                            }
                        }
                        // the steps exchange data through LDS only; global traffic crosses
                        // between the groups at phase boundaries (full barrier above)
                        lds_barrier();
                    }
                    // last recomputed step of segment jB (its sum is in psum since the last barrier)
                    if (rec && LB > 0) {
                        if (LB == 1)
                            store_entry0(jB);
                        else
                            finish(jB, t0B + LB - 1);
                    }
                }
                if (!rec) {
                    flush_pending();
                    if (rank_has_prev) ranktab[rank_prev >> 1] = 0u;  // the last step (t = 0) used half 0
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = 16 * w + 4 * g + v;
                        if (i < N) add_fixed(&a.pi64[(size_t)k * N + i], gpi[v], F, &a.nanflag[k]);
                    }
                    if (lane_nan) atomicOr(&a.nanflag[k], 1);
                }
                // this tile's n_A = A o C for this wave's rows and half of the columns (row
                // base opaque: the flush's addresses are not kept live across the tile loop)
                {
                    const int rb = opaque(k * N + 16 * w + 4 * g);
                    const int ib = 16 * w + 4 * g;
#pragma unroll
                    for (int rj = 0; rj < RH; ++rj)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int jj = 16 * (rj0 + rj) + sl;
                            const size_t e = (size_t)(rb + v) * N + jj;
                            if (ib + v < N && jj < N) add_fixed(&a.A64[e], d.A[e] * C[rj][v], F, &a.nanflag[k]);
                        }
                }
                }  // Tmax > 0
                // the tile's emission partial into its slab slot (zeros for an empty tile)
                __syncthreads();
                const int64_t slot = slab_slot(gbeg, k, tile);
                float *dst = a.slab + (size_t)(dbg_in(slot, slab_slots(a.S, a.K), HMM_DEBUG_SLAB) ? slot : 0) * M * NP;
                for (int idx = threadIdx.x; idx < M * NP; idx += blockDim.x) {
                    const int o = idx / NP, ic = idx % NP;
                    dst[(size_t)o * NP + (ic ^ (o * 4 & swz))] = nbl[idx];
                    nbl[idx] = 0.0f;
                }
            }
        }
    }
}

constexpr size_t COOP_LDS_LIMIT = 160 * 1024;

// Dynamic LDS of the partial variant: the [M][NP] partial, then the [2][ceil(M / 2)] slot-mask table.
template <int R>
size_t nb_lds_bytes(int M) {
    return ((size_t)M * 16 * R * 4 + (size_t)2 * ((M + 1) / 2) * 4 + 15) / 16 * 16;
}

// The LDS partial serves one-block waves (up to 128 states) whose partial fits,
// when the slab of per-tile partials stays within SLAB_MAX_BYTES.
template <int R>
bool use_nb_lds(int M, int S, int K) {
    constexpr int BO = adj_bo(R);
    if (BO > 1) return false;
    if (slab_slots(S, K) * M * 16 * R * 4 > SLAB_MAX_BYTES) return false;
    return nb_lds_bytes<R>(M) + AdjCoopShape<R, BO>::small_bytes + 64 <= COOP_LDS_LIMIT;
}

// The pipelined kernel serves 64-state tiles whose LDS partial fits next to
// its buffers.  (With 6 or 8 blocks its 12 or 16 waves leave fewer than 170
// registers per wave, and the step spills.)
template <int R>
bool use_pipe(int M, int S, int K) {
    if constexpr (R != 4) {
        return false;
    } else {
        using SH = AdjCoopShape<R, 1>;
        if (slab_slots(S, K) * M * 16 * R * 4 > SLAB_MAX_BYTES) return false;
        const size_t small = (SH::xch_floats + SH::w_floats + 2 * SH::at_floats) * 4 + 2 * PACH * TILE * 4 + TILE * 4;
        return nb_lds_bytes<R>(M) + small + 64 <= COOP_LDS_LIMIT;
    }
}

template <int R>
int grid_pipe(int M, int cu_count, int K) {
    if constexpr (R != 4) {
        return 0;
    } else {
        auto kern = k_adj_pipe<R>;
        const size_t dyn = nb_lds_bytes<R>(M);
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 2 * R * WAVE, dyn) != hipSuccess || per_cu < 1)
            per_cu = 1;
        int grid = cu_count * per_cu;
        if (K > 0 && grid >= K) grid = (grid / K) * K;
        return grid;
    }
}

template <int R, bool NBLDS, bool FULL = false>
int grid_t(int M, int cu_count, int K) {
    constexpr int BO = adj_bo(R);
    if constexpr (NBLDS && BO > 1) return 0;  // not instantiated: the partial serves one-block waves
    auto kern = k_adj_coop<R, BO, NBLDS && BO == 1, (BO > 1), FULL>;
    const size_t dyn = NBLDS ? nb_lds_bytes<R>(M) : 0;
    if (dyn > 0) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, R / BO * WAVE, dyn) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int grid = cu_count * per_cu;
    if (K > 0 && grid >= K) grid = (grid / K) * K;
    return grid;
}

template <int R>
int grid_r(int M, int S, int cu_count, int K) {
    if (use_pipe<R>(M, S, K)) return grid_pipe<R>(M, cu_count, K);
    return use_nb_lds<R>(M, S, K) ? grid_t<R, true>(M, cu_count, K) : grid_t<R, false>(M, cu_count, K);
}

template <int R>
hipError_t launch_r(const DevPtrs &d, const AdjLaunch &a, int cu_count, hipStream_t st) {
    constexpr int BO = adj_bo(R);
    constexpr bool STREAM = BO > 1;
    if (STREAM && a.frag == nullptr) return hipErrorInvalidValue;
    const int grid =
        persistent_grid(grid_r<R>(a.M, a.S, cu_count, a.K), tile_bound(a.S, a.K, false, TILE), 1, a.K, a.max_grid);
    if (grid > a.seg_slots) return hipErrorInvalidValue;
    // Full storage possible: its walk runs first and exits unless the rows of
    // every sequence fit; the checkpoint kernel below exits when they do.  The
    // walk keeps the emission counts where the checkpoint kernel of the shape
    // keeps them (LDS partial and slab, or the global sums).
    if (a.arow != nullptr) {
        const bool slab_shape = use_pipe<R>(a.M, a.S, a.K) || (!STREAM && use_nb_lds<R>(a.M, a.S, a.K));
        if (slab_shape && (STREAM || a.slab == nullptr)) return hipErrorInvalidValue;
        if (!slab_shape && a.B64 == nullptr) return hipErrorInvalidValue;
        if constexpr (!STREAM) {
            if (slab_shape) {
                const int gf = persistent_grid(grid_t<R, true, true>(a.M, cu_count, a.K), tile_bound(a.S, a.K, false, TILE),
                                               1, a.K, a.max_grid);
                k_adj_coop<R, BO, true, false, true><<<gf, R / BO * WAVE, nb_lds_bytes<R>(a.M), st>>>(d, a);
            }
        }
        if (!slab_shape) {
            const int gf = persistent_grid(grid_t<R, false, true>(a.M, cu_count, a.K), tile_bound(a.S, a.K, false, TILE),
                                           1, a.K, a.max_grid);
            k_adj_coop<R, BO, false, STREAM, true><<<gf, R / BO * WAVE, 0, st>>>(d, a);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if constexpr (R == 4) {
        if (use_pipe<R>(a.M, a.S, a.K)) {
            if (a.slab == nullptr) return hipErrorInvalidValue;
            k_adj_pipe<R><<<grid, 2 * R * WAVE, nb_lds_bytes<R>(a.M), st>>>(d, a);
            return hipGetLastError();
        }
    }
    if constexpr (!STREAM) {
        if (use_nb_lds<R>(a.M, a.S, a.K)) {
            if (a.slab == nullptr) return hipErrorInvalidValue;
            k_adj_coop<R, BO, true, false, false><<<grid, R / BO * WAVE, nb_lds_bytes<R>(a.M), st>>>(d, a);
            return hipGetLastError();
        }
    }
    if (a.B64 == nullptr) return hipErrorInvalidValue;
    k_adj_coop<R, BO, false, STREAM, false><<<grid, R / BO * WAVE, 0, st>>>(d, a);
    return hipGetLastError();
}

// ---- Emission counts from the stored gamma rows.  A position whose rows hold
// gamma is one the backward pass walked with a finite likelihood (its "act"):
// a valid sequence with steps, a valid model and flag 0.  Buckets are (model,
// symbol); the rows of a bucket are summed as 64-bit fixed-point values, the
// same values the per-step atomics add, so the counts are the same bit for bit
// whatever order the rows take in their bucket.
__device__ __forceinline__ bool gamma_rows_of(const DevPtrs &d, const AdjLaunch &a, int p, int *mk, int32_t *T,
                                              int64_t *off) {
    const int seq = a.perm[p];
    *T = d.lengths[seq];
    *off = d.offsets[seq];
    *mk = d.model_of_seq[seq];
    const bool bad = seq_bad(*T, *off, a.max_len, a.total) || *mk < 0 || *mk >= a.K;
    return !bad && *T > 0 && a.flag[p] == 0;
}

// One wave per position: the rows of each bucket.
__global__ void __launch_bounds__(256) k_grows_hist(DevPtrs d, AdjLaunch a) {
    if (!grad_full(a.arow, a.rowpos, a.S, a.grad_rows)) return;
    const int p = (int)(blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    int mk;
    int32_t T;
    int64_t off;
    if (p >= a.S || !gamma_rows_of(d, a, p, &mk, &T, &off)) return;
    for (int t = lane; t < T; t += WAVE) {
        const int o = d.symbols[off + t];
        atomicAdd(&a.cursor[(size_t)mk * a.M + ((unsigned)o < (unsigned)a.M ? o : 0)], 1);
    }
}

// One workgroup: bucket[b] = rows of the buckets before b, bucket[KM] = all;
// the counts become the scatter cursors.
__global__ void __launch_bounds__(1024) k_grows_scan(AdjLaunch a, int nb) {
    if (!grad_full(a.arow, a.rowpos, a.S, a.grad_rows)) return;
    __shared__ int32_t part[1024];
    const int per = (nb + 1023) / 1024;
    const int e0 = min(nb, (int)threadIdx.x * per), e1 = min(nb, e0 + per);
    int32_t local = 0;
    for (int e = e0; e < e1; ++e) local += a.cursor[e];
    part[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t y = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - local;
    for (int e = e0; e < e1; ++e) {
        const int32_t c = a.cursor[e];
        a.bucket[e] = run;
        a.cursor[e] = run;
        run += c;
    }
    if (threadIdx.x == 1023) a.bucket[nb] = part[1023];
}

// One wave per position: each row index into its bucket.
__global__ void __launch_bounds__(256) k_grows_scatter(DevPtrs d, AdjLaunch a) {
    if (!grad_full(a.arow, a.rowpos, a.S, a.grad_rows)) return;
    const int p = (int)(blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    int mk;
    int32_t T;
    int64_t off;
    if (p >= a.S || !gamma_rows_of(d, a, p, &mk, &T, &off)) return;
    const int64_t rb = a.rowpos[p];
    const int64_t nrows = a.bucket[(size_t)a.K * a.M];
    for (int t = lane; t < T; t += WAVE) {
        const int o = d.symbols[off + t];
        const int slot = atomicAdd(&a.cursor[(size_t)mk * a.M + ((unsigned)o < (unsigned)a.M ? o : 0)], 1);
        if (dbg_in(slot, nrows, HMM_DEBUG_GRAD_ROWS)) a.srows[slot] = (uint32_t)(rb + t);
    }
}

// One wave per bucket (model k, symbol o): its rows' gamma, lane l holding
// states 4 l .. 4 l + 3, into the symbol-major fixed-point counts.
__global__ void __launch_bounds__(256) k_grows_reduce(AdjLaunch a) {
    if (!grad_full(a.arow, a.rowpos, a.S, a.grad_rows)) return;
    const int b = (int)(blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    const int NP = a.NP;
    if (b >= a.K * a.M || 4 * lane >= NP) return;
    const int F = fixed_exponent(*a.wmax, a.S, a.max_len);
    const int e0 = a.bucket[b], e1 = a.bucket[b + 1];
    unsigned long long acc[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll 4
    for (int e = e0; e < e1; ++e) {
        int64_t r = a.srows[e];
        if (!dbg_in(r, a.grad_rows, HMM_DEBUG_GRAD_ROWS)) r = 0;
        const float4 q = *(const float4 *)&a.arow[(size_t)r * NP + 4 * lane];
        const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float gm = qv[v];
            acc[v] += to_fixed(__builtin_isfinite(gm) ? gm : 0.0f, F);
        }
    }
    unsigned long long *dst = a.B64 + (size_t)b * NP;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * lane + v;
        dst[quad_t(i)] = i < a.N ? acc[v] : 0ull;
    }
}

// Streamed fragments of model k: set 0 (A_k^T, recompute) and set 1 (A_k,
// beta), float4 index (((set * NW + w) * R + rp) * 64 + lane) * BO + b with
// components v = 0..3:
//   set 0: A_k[16 rp + 4 g + v][16 (BO w + b) + sl],  set 1: A_k[16 (BO w + b) + sl][16 rp + 4 g + v]
// (g = lane / 16, sl = lane % 16; zero outside N x N).
__global__ void k_coop_frags(const float *A, float4 *frag, int N, int R, int BO) {
    const int k = blockIdx.y;
    const size_t per_model = (size_t)2 * R * R * WAVE;  // float4
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per_model) return;
    const int NW = R / BO;
    const int b = (int)(idx % BO);
    const int lane = (int)((idx / BO) % WAVE);
    const int rp = (int)((idx / ((size_t)BO * WAVE)) % R);
    const int w = (int)((idx / ((size_t)BO * WAVE * R)) % NW);
    const int set = (int)(idx / ((size_t)BO * WAVE * R * NW));
    const int g = lane >> 4, sl = lane & 15;
    const float *Ak = A + (size_t)k * N * N;
    float v4[4];
    for (int v = 0; v < 4; ++v) {
        const int i = set == 0 ? 16 * rp + 4 * g + v : 16 * (BO * w + b) + sl;
        const int j = set == 0 ? 16 * (BO * w + b) + sl : 16 * rp + 4 * g + v;
        v4[v] = (i < N && j < N) ? Ak[(size_t)i * N + j] : 0.0f;
    }
    frag[(size_t)k * per_model + idx] = float4{v4[0], v4[1], v4[2], v4[3]};
}

}  // namespace

bool adj_coop_supported(int NP) { return NP >= 64 && NP <= 256 && NP % 32 == 0; }

bool adj_coop_streams(int NP) { return adj_bo(NP / 16) > 1; }

int adj_coop_slots(int NP, int M, int S, int K, int cu_count) {
    switch (NP / 16) {
        case 4: return grid_r<4>(M, S, cu_count, K);
        case 6: return grid_r<6>(M, S, cu_count, K);
        case 8: return grid_r<8>(M, S, cu_count, K);
        case 10: return grid_r<10>(M, S, cu_count, K);
        case 12: return grid_r<12>(M, S, cu_count, K);
        case 14: return grid_r<14>(M, S, cu_count, K);
        case 16: return grid_r<16>(M, S, cu_count, K);
        default: return 0;
    }
}

bool adj_coop_pipelined(int NP, int M, int S, int K) {
    switch (NP / 16) {
        case 4: return use_pipe<4>(M, S, K);
        default: return false;
    }
}

bool adj_coop_slab(int NP, int M, int S, int K) {
    switch (NP / 16) {
        case 4: return use_pipe<4>(M, S, K) || use_nb_lds<4>(M, S, K);
        case 6: return use_nb_lds<6>(M, S, K);
        case 8: return use_nb_lds<8>(M, S, K);
        default: return false;
    }
}

int64_t adj_coop_seg_stride(int NP, int M, int S, int K, int max_len) {
    int L = 1;
    while ((int64_t)L * L < max_len) ++L;
    const int R = NP / 16, BO = adj_bo(R);
    // float4 alphahat per owned block + e + o, per lane and wave; two halves
    // (segment parity) for the pipelined kernel
    return (int64_t)L * (R / BO) * WAVE * (4 * BO + 2) * (adj_coop_pipelined(NP, M, S, K) ? 2 : 1);
}

void launch_coop_frags(const float *A, float *frag, int K, int N, int NP, hipStream_t st) {
    const int R = NP / 16, BO = adj_bo(R);
    const size_t per_model = (size_t)2 * R * R * WAVE;
    dim3 grid((unsigned)((per_model + 255) / 256), (unsigned)K);
    hipLaunchKernelGGL(k_coop_frags, grid, dim3(256), 0, st, A, (float4 *)frag, N, R, BO);
}

hipError_t launch_adj_coop(const DevPtrs &d, const AdjLaunch &a, int cu_count, hipStream_t st) {
    switch (a.NP / 16) {
        case 4: return launch_r<4>(d, a, cu_count, st);
        case 6: return launch_r<6>(d, a, cu_count, st);
        case 8: return launch_r<8>(d, a, cu_count, st);
        case 10: return launch_r<10>(d, a, cu_count, st);
        case 12: return launch_r<12>(d, a, cu_count, st);
        case 14: return launch_r<14>(d, a, cu_count, st);
        case 16: return launch_r<16>(d, a, cu_count, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_counts_from_rows(const DevPtrs &d, const AdjLaunch &a, hipStream_t st) {
    if (a.srows == nullptr || a.S == 0) return hipSuccess;
    if (a.B64 == nullptr || a.NP > 4 * WAVE) return hipErrorInvalidValue;
    const int nb = a.K * a.M;
    launch_fill_i32(a.cursor, (size_t)nb, 0, st);
    const unsigned pos_blocks = (unsigned)((a.S + 3) / 4);
    hipLaunchKernelGGL(k_grows_hist, dim3(pos_blocks), dim3(256), 0, st, d, a);
    hipLaunchKernelGGL(k_grows_scan, dim3(1), dim3(1024), 0, st, a, nb);
    hipLaunchKernelGGL(k_grows_scatter, dim3(pos_blocks), dim3(256), 0, st, d, a);
    hipLaunchKernelGGL(k_grows_reduce, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

HMM_DEBUG_TAKE(debug_take_adj_coop)

}  // namespace hmm
