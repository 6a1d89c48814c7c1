// Cooperative-tile forward kernel (gfx950) for large state counts: the dense
// grouped step of the recognition path when one wave cannot hold A_k.
//
// Same recursion as the per-wave kernel (paper Sec. 2.7 "Forward", one HMM
// per action evaluated independently, Sec. 3 item 3), distributed over a
// workgroup of R / BO waves (R = NP / 16 state blocks, BO blocks per wave) per
// tile of 16 length-sorted sequences of one model (see coop_step.cuh for the
// data movement).  Per step and workgroup: 4 R^2 MFMAs of 16x16x4 FP32, one
// barrier, one exchange of 16 x NP floats through LDS.  Emission rows B^T[o][.] come from L2 (B^T of one model is up to
// 1 MiB and stays resident in its XCD's L2); the symbol and row of step t+1
// are fetched during step t.  The gradient's variant (CKPT) keeps alphahat for
// the backward pass: every step's row and exponent when the workspace's rows
// hold the batch (decided on the device from the row prefix), else a
// checkpoint every ceil(sqrt(Tmax)) steps.
#include <climits>

#include "common.cuh"
#include "coop_step.cuh"
#include "kernels.h"

namespace hmm {
namespace {

constexpr int CCH = 32;  // symbols per staging chunk

template <int R, int BO, bool CKPT>
__global__ void __launch_bounds__(R / BO * WAVE) k_fwd_coop(DevPtrs d, FwdLaunch f) {
    using SH = CoopShape<R>;
    constexpr int NP = SH::NP;
    constexpr int XROW = SH::XROW;
    __shared__ __align__(16) float xch[SH::floats];
    __shared__ int32_t sym[2][CCH * TILE];
    __shared__ int32_t tile_sh;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int r0 = BO * w;                   // first owned 16-state block
    const int sl = lane & 15, g = lane >> 4;
    const int K = f.K, N = f.N, M = f.M;
    float *xbuf = xch;                       // [2][16][XROW]
    float *psum = xch + SH::x_floats;        // [2][R][16]
    // full-storage gradient: every step's alphahat in place of the checkpoints
    const bool full = CKPT && grad_full(f.arow, f.rowpos, f.S, f.grad_rows);

    const int G = gridDim.x;
    const int k_first = G >= K ? (int)(blockIdx.x % K) : (int)blockIdx.x;
    const int k_step = G >= K ? K : G;
    for (int k = k_first; k < K; k += k_step) {
        const int grp = f.all_pairs ? 0 : k;
        const int gbeg = f.gstart[grp], gend = f.gstart[grp + 1];
        const int ntiles = (gend - gbeg + TILE - 1) / TILE;
        if (ntiles == 0) continue;
        const float *btk = f.bt + (size_t)k * M * NP;
        const float *pik = d.pi + (size_t)k * N;
        float af[BO][R][4];
        coop_load_fwd_fragments<R, BO>(af, d.A + (size_t)k * N * N, N, r0, g, sl);

        for (;;) {
            if (threadIdx.x == 0) tile_sh = atomicAdd(&f.queue[k], 1);
            __syncthreads();
            const int tile = __builtin_amdgcn_readfirstlane(tile_sh);  // scalar exit: the loop holds barriers
            __syncthreads();
            if (tile >= ntiles) break;

            const int pos = gbeg + tile * TILE + sl;
            const bool has = pos < gend;
            const int seq = has ? f.perm[pos] : 0;
            int32_t T = 0;
            int64_t off = 0;
            bool bad = false;
            if (has) {
                T = d.lengths[seq];
                off = d.offsets[seq];
                bad = seq_bad(T, off, f.max_len, f.total);
                if (!f.all_pairs) {
                    const int mk = d.model_of_seq[seq];
                    bad |= (mk < 0 || mk >= K);
                }
                if (bad) T = 0;
            }
            const int Tmax = __builtin_amdgcn_readfirstlane(wave_max_int(T));
            if (Tmax == 0) {
                if (has && g == 0 && w == 0) {
                    store_ll(f, seq, pos, k, bad ? NAN : 0.0f);
                    if (bad) atomicMin(f.err, seq);
                    if (CKPT) f.flag[pos] = bad ? 1 : 0;
                }
                continue;
            }
            int L = 1;
            if (CKPT && !full)
                while (L * L < Tmax) ++L;
            const int64_t rb = (full && T > 0) ? f.rowpos[pos] : 0;  // first stored row of the sequence
            // symbols: wave 0 stages chunks (register prefetch, chunk c lives in sym[c & 1])
            const int32_t *sbase = T > 0 ? d.symbols + off : d.symbols;
            const int tlim = T > 0 ? T - 1 : 0;
            int32_t nxt[CCH / 4];
            auto load_chunk = [&](int t0) {
#pragma unroll
                for (int u = 0; u < CCH / 4; ++u) nxt[u] = sbase[min(t0 + 4 * u + g, tlim)];
            };
            auto store_chunk = [&](int c) {
#pragma unroll
                for (int u = 0; u < CCH / 4; ++u) sym[c & 1][u * WAVE + lane] = nxt[u];
            };
            auto read_sym = [&](int t) {
                const int pp = t % CCH;
                return sym[(t / CCH) & 1][(pp / 4) * WAVE + 16 * (pp % 4) + sl];
            };
            if (w == 0) {
                load_chunk(0);
                store_chunk(0);
                load_chunk(CCH);
                store_chunk(1);
            }
            __syncthreads();

            bool symbad = false;
            int o = read_sym(0);
            symbad |= (0 < T) && (o < 0 || o >= M);
            o = ((unsigned)o < (unsigned)M) ? o : 0;
            float4 bA[BO], bB[BO];
#pragma unroll
            for (int b = 0; b < BO; ++b) bA[b] = *(const float4 *)&btk[(size_t)o * NP + 16 * (r0 + b) + 4 * g];
            float x[BO][4] = {};
            int E = 0, E_end = 0;
            float c_end = 1.0f;
            int ck_t = 0, ck_c = 0;  // next checkpointed step and its index
            // Read phase of step t: finishes step t - 1 (its sum, exponent and
            // checkpoint) and returns that step's exponent (0 at t = 0).
            auto read_phase = [&](int t) -> int {
                int e = 0;
                if (t > 0) {
                    const float cs = coop_step_sum<R>(psum + ((t - 1) & 1) * R * TILE, sl);
                    e = frexp_exp(cs);
                    if (t - 1 == T - 1) {
                        E_end = E;
                        c_end = cs;
                    }
                    E += e;
                    if (full) {
                        if (t - 1 < T) {
                            const int64_t row = rb + (t - 1);
                            if (dbg_in(row, f.grad_rows, HMM_DEBUG_GRAD_ROWS)) {
#pragma unroll
                                for (int b = 0; b < BO; ++b) {
                                    float *dst = f.arow + (size_t)row * NP + 16 * (r0 + b) + 4 * g;
                                    *(float4 *)dst = float4{ldexp_f(x[b][0], -e), ldexp_f(x[b][1], -e),
                                                            ldexp_f(x[b][2], -e), ldexp_f(x[b][3], -e)};
                                }
                                if (w == 0 && g == 0) f.aexp[row] = e;
                            }
                            if (t - 1 == T - 1 && w == 0 && g == 0) f.mlast[pos] = ldexp_f(cs, -e);
                        }
                    } else if (CKPT && t - 1 == ck_t) {  // t - 1 = L ck_c
                        if (t - 1 < T && dbg_in(ck_c, f.nck, HMM_DEBUG_CKPT)) {
#pragma unroll
                            for (int b = 0; b < BO; ++b) {
                                float *dst = f.ckpt + ((size_t)pos * f.nck + ck_c) * NP + 16 * (r0 + b) + 4 * g;
                                *(float4 *)dst = float4{ldexp_f(x[b][0], -e), ldexp_f(x[b][1], -e),
                                                        ldexp_f(x[b][2], -e), ldexp_f(x[b][3], -e)};
                            }
                            if (w == 0 && g == 0) f.ckexp[(size_t)pos * f.nck + ck_c] = e;
                        }
                        ck_t += L;
                        ++ck_c;
                    }
                }
                return e;
            };
            // Step t < Tmax: read phase, then the compute phase.
            // bcur holds the emission rows of step t, bnext receives
            // those of step t + 1.  The loop below alternates the two register
            // sets, so no copy carries a pending load across the loop latch (the
            // compiler would wait for every outstanding load there); the load
            // into bnext is issued every step (a valid row when t + 1 = Tmax) so
            // that the wait before its use in the next step can count it.
            // The symbol of step s is read from LDS at step s - 2 (o2), so that the
            // emission rows of step t + 1 (symbol o1, any value at t + 1 = Tmax,
            // clamped below) are requested before anything else of step t.
            // Chunk c + 1 >= 2 is loaded by wave 0 at step 32 c (always the first
            // step of a pair) and stored at step 32 c + 1 (the second), into the
            // buffer of chunk c - 1, whose last reader, step 32 c - 3, every wave
            // has passed; the barrier of step 32 c + 1 publishes it long before
            // its first reader, step 32 c + 30.  Loading and storing inside one
            // iteration keeps the staging registers out of the loop latch.
            auto step = [&](int t, const float4 (&bcur)[BO], float4 (&bnext)[BO], int o1, int &o2, bool chunk_ld,
                            bool chunk_st) {
                int on = o1;
                symbad |= (t + 1 < T) && (on < 0 || on >= M);
                on = ((unsigned)on < (unsigned)M) ? on : 0;
#pragma unroll
                for (int b = 0; b < BO; ++b) bnext[b] = *(const float4 *)&btk[(size_t)on * NP + 16 * (r0 + b) + 4 * g];
                // first operand of this step's product, requested with the block sums
                const float *xprev = xbuf + ((t - 1) & 1) * TILE * XROW;
                const float4 q0 = *(const float4 *)&xprev[sl * XROW + 4 * g];
                const int e = read_phase(t);
                if (chunk_ld) load_chunk(t + CCH);
                o2 = read_sym(t + 2);
                floatx4 u[BO];
                if (t == 0) {
#pragma unroll
                    for (int b = 0; b < BO; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = 16 * (r0 + b) + 4 * g + v;
                            u[b][v] = i < N ? pik[i] : 0.0f;
                        }
                } else {
                    coop_matvec_q0<R, BO>(af, xprev, q0, e, g, sl, u);
                }
#pragma unroll
                for (int b = 0; b < BO; ++b) {
                    const float part = coop_emit(u[b], bcur[b], x[b]);
                    *(float4 *)&xbuf[(t & 1) * TILE * XROW + sl * XROW + 16 * (r0 + b) + 4 * g] =
                        float4{x[b][0], x[b][1], x[b][2], x[b][3]};
                    if (g == 0) psum[(t & 1) * R * TILE + (r0 + b) * TILE + sl] = part;
                }
                if (chunk_st) store_chunk(t / CCH + 1);
                // the waves exchange alphahat through LDS only: the emission rows and
                // symbols requested for the next steps stay in flight across the barrier
                lds_barrier();
            };
            int oA = 0, oB = read_sym(1);  // symbols of the next even and odd steps
            int t = 0;
            for (; t + 1 < Tmax; t += 2) {
                const bool chunk = w == 0 && t > 0 && (t % CCH) == 0;
                step(t, bA, bB, oB, oA, chunk, false);
                step(t + 1, bB, bA, oA, oB, false, chunk);
            }
            if (t < Tmax) step(t++, bA, bB, oB, oA, false, false);
            read_phase(t);
            if (has && g == 0 && w == 0) {
                float r = (float)((double)E_end * LN2 + (double)logf(c_end));
                if (bad || symbad) r = NAN;
                store_ll(f, seq, pos, k, r);
                if (bad || symbad) atomicMin(f.err, seq);
                if (CKPT) f.flag[pos] = (r > -INFINITY && r < INFINITY) ? 0 : 1;
            }
            __syncthreads();
        }
    }
}

// Blocks per wave: one up to 8 blocks (N <= 128), two above, so that a lane's
// fragments (4 R BO floats) fit the register budget of the workgroup size.
template <int R>
constexpr int coop_bo() { return R > 8 ? 2 : 1; }

template <int R, bool CKPT>
hipError_t launch_t(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st) {
    constexpr int BO = coop_bo<R>();
    auto kern = k_fwd_coop<R, BO, CKPT>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, R / BO * WAVE, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const int grid = persistent_grid(cu_count * per_cu, tile_bound(f.S, f.K, f.all_pairs, TILE), 1, f.K, f.max_grid);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(R / BO * WAVE), 0, st, d, f);
    return hipGetLastError();
}

}  // namespace

bool fwd_coop_supported(int NP) { return NP >= 64 && NP <= 256 && NP % 32 == 0; }

hipError_t launch_fwd_coop(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st) {
    const bool ck = f.ckpt != nullptr;
#define HMM_COOP_CASE(R) \
    case R:              \
        return ck ? launch_t<R, true>(d, f, cu_count, st) : launch_t<R, false>(d, f, cu_count, st);
    switch (f.NP / 16) {
        HMM_COOP_CASE(4)
        HMM_COOP_CASE(6)
        HMM_COOP_CASE(8)
        HMM_COOP_CASE(10)
        HMM_COOP_CASE(12)
        HMM_COOP_CASE(14)
        HMM_COOP_CASE(16)
        default:
            return hipErrorInvalidValue;
    }
#undef HMM_COOP_CASE
}

HMM_DEBUG_TAKE(debug_take_fwd_coop)

}  // namespace hmm
