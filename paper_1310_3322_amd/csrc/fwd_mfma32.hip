// Batched forward kernel on 32x32x2 FP32 MFMA (gfx950): tiles of 32 sequences.
//
// Same recursion and work distribution as fwd_mfma.hip (paper Sec. 2.7
// "Forward"; the HMMs of the actions are independent, Sec. 3 item 3), with 32
// length-sorted sequences of one model per wave.  The 32x32x2 result tile
// gives each lane one sequence (lane % 32) and sixteen states of each 32-state
// block r: 32 r + 8 (v / 4) + 4 (lane / 32) + v % 4, v = 0..15.  As in the
// 16-sequence kernel the k-step (block r', register v) feeds half h = lane / 32
// exactly the state its lanes hold in register v, so step t's results are step
// t+1's B operand.  Per step a wave issues 16 R^2 MFMAs of 64 cycles against
// the same per-sequence epilogue (emission product, one cross-half sum,
// exponent, rescale), which halves the vector work per MFMA cycle compared with
// 16-sequence tiles.  Used for recognition and log-likelihoods when tiles are
// plentiful; the gradient keeps the 16-sequence kernels.
#include <climits>
#include <type_traits>
#include <type_traits>

#include "common.cuh"
#include "kernels.h"

namespace hmm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int T32 = 32;              // sequences per tile
constexpr int CH32 = 16;             // symbols per staging chunk (8 per lane)
constexpr int SYM32 = CH32 * T32;    // symbols per wave buffer
constexpr int WAVES32 = 4;           // waves per workgroup

// B^T rows in LDS, row o at byte o * row_stride32(NP): a row of NP floats and 16
// bytes of padding.  With the padding, the float4 chunk c of row o starts in bank
// group (o (NP / 4 + 1) + c) mod 16 of the 16 groups of four 4-byte banks, so the
// 16 lanes of one 16-byte LDS pass, which read one chunk of 16 random rows, spread
// over all 16 groups; a lane's chunks of one row are at fixed offsets from the
// row's start, which takes one address computation per step.
__host__ __device__ constexpr int row_stride32(int NP) { return NP * 4 + 16; }

// With one 32-state block (R = 1) the step fits 128 VGPRs, which allows four
// waves per SIMD; R = 2 needs about twice that.
template <int R, bool BLDS>
__global__ void __launch_bounds__(WAVES32 * WAVE) __attribute__((amdgpu_waves_per_eu(R == 1 ? 4 : 1, 8)))
k_fwd_mfma32(DevPtrs d, FwdLaunch f) {
    constexpr int NP = 32 * R;
    extern __shared__ __align__(16) unsigned char smem[];
    // 16-bit symbols when B^T fits in LDS (M <= 1024 there), which leaves room for the
    // padded rows at four workgroups per CU
    typedef typename std::conditional<BLDS, uint16_t, int32_t>::type sym_t;
    __shared__ sym_t sym_all[WAVES32 * SYM32];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int sl = lane & 31;        // sequence slot
    const int h = lane >> 5;         // half: states 32 r + 8 q + 4 h + 0..3
    const int K = f.K, N = f.N, M = f.M;
    unsigned char *btl = smem;
    sym_t *sym = sym_all + wave * SYM32;

    // Scoring all pairs, the tiles are split over the XCDs (workgroup b runs on
    // XCD b mod 8): slice x takes one tile of every group of 8 consecutive tiles
    // of every model, so each tile's symbols are read into one XCD's L2 and serve
    // all the models there.  The tiles come longest first; the slice takes the
    // x-th tile from the front of even groups and from the back of odd ones, so
    // the slices' shares of work differ by at most one group's spread instead of
    // the sum of them.  Own-model calls keep one model per workgroup.
    const int XS = xcd_slices(f.all_pairs && !(f.tune_flags & HMM_TUNE_XCD_OFF), gridDim.x, K);
    const int x = (int)(blockIdx.x % XS);
    const int G = (int)gridDim.x / XS, gi = (int)blockIdx.x / XS;
    const int k_first = G >= K ? gi % K : gi;
    const int k_step = G >= K ? K : G;
    for (int k = k_first; k < K; k += k_step) {
        const int grp = f.all_pairs ? 0 : k;
        const int gbeg = f.gstart[grp], gend = f.gstart[grp + 1];
        const int ntiles_all = (gend - gbeg + T32 - 1) / T32;
        const int full = ntiles_all / XS, rem = ntiles_all % XS;
        const int ntiles = full + (((full & 1) ? XS - 1 - x : x) < rem ? 1 : 0);  // this slice's tiles
        const float *btk = f.bt + (size_t)k * M * NP;
        if (BLDS) {
            __syncthreads();
            const int n4 = M * NP / 4;
            for (int i = threadIdx.x; i < n4; i += blockDim.x) {
                const int o = i / (NP / 4), c = i % (NP / 4);
                *(float4 *)(btl + o * row_stride32(NP) + 16 * c) = ((const float4 *)btk)[i];
            }
            __syncthreads();
        }
        if (ntiles == 0) continue;
        // A operand fragments: af[r][rp][v] = A_k[32 rp + 8 (v/4) + 4 h + v%4][32 r + sl]
        float af[R][R][16];
        {
            const float *Ak = d.A + (size_t)k * N * N;
            const int lane_off = opaque(4 * h * N + sl);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int rp = 0; rp < R; ++rp)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int i = 32 * rp + 8 * (v / 4) + 4 * h + v % 4, j = 32 * r + sl;
                        af[r][rp][v] =
                            (i < N && j < N) ? Ak[lane_off + (32 * rp + 8 * (v / 4) + v % 4) * N + 32 * r] : 0.0f;
                    }
        }
        const float *pik = d.pi + (size_t)k * N;
        // Rescaling every other step is safe when every emission probability of the
        // model is at least 2^-60: a step then multiplies the sum of a normalised
        // alpha by at least 2^-61 (rows of A sum to 1), so two steps keep it above
        // 2^-122, in the normal range.
        const bool lazy = f.bmin != nullptr && __uint_as_float(f.bmin[k]) >= 8.673617379884035e-19f;

        for (;;) {
            const int jt = wave_pop(&f.queue[k * XS + x]);
            if (jt >= ntiles) break;
            const int tile = XS * jt + ((jt & 1) ? XS - 1 - x : x);

            const int pos = gbeg + tile * T32 + sl;
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
            const int Tmin = __builtin_amdgcn_readfirstlane(-wave_max_int(T > 0 ? -T : INT_MIN + 1));
            // Symbol chunks: nxt[u] = symbol of sequence sl at step t0 + 8 h + u (the
            // lane's half of the chunk, consecutive, so that a chunk inside the
            // sequence takes one address; the steps past its end repeat the last
            // symbol), stored as sym[u][lane]; checked and clamped when a chunk
            // enters LDS.
            const int32_t *sbase = T > 0 ? d.symbols + off : d.symbols;
            const int tlim = T > 0 ? T - 1 : 0;
            int32_t nxt[CH32 / 2];
            bool symbad = false;
            auto load_chunk = [&](int t0) {
                const int tb = t0 + (CH32 / 2) * h;
                if (__builtin_amdgcn_ballot_w64(tb + CH32 / 2 - 1 > tlim) == 0) {  // every lane's half inside
                    // two 16-byte loads (symbols are 4-byte aligned; global loads take any
                    // 4-byte-aligned address)
                    int4 v0, v1;
                    __builtin_memcpy(&v0, sbase + tb, 16);
                    __builtin_memcpy(&v1, sbase + tb + 4, 16);
                    nxt[0] = v0.x; nxt[1] = v0.y; nxt[2] = v0.z; nxt[3] = v0.w;
                    nxt[4] = v1.x; nxt[5] = v1.y; nxt[6] = v1.z; nxt[7] = v1.w;
                } else {
#pragma unroll
                    for (int u = 0; u < CH32 / 2; ++u) nxt[u] = sbase[min(tb + u, tlim)];
                }
            };
            auto store_chunk = [&](int t0) {
                wave_lds_sync();
#pragma unroll
                for (int u = 0; u < CH32 / 2; ++u) {
                    const int o = nxt[u];
                    const bool ok = (unsigned)o < (unsigned)M;
                    symbad |= (t0 + (CH32 / 2) * h + u < T) && !ok;
                    sym[u * WAVE + lane] = (sym_t)(ok ? o : 0);
                }
                wave_lds_sync();
            };
            auto read_sym = [&](int t) {
                const int pp = t % CH32;
                return sym[(pp % (CH32 / 2)) * WAVE + 32 * (pp / (CH32 / 2)) + sl];
            };
            auto gather = [&](int o, float4 (&b)[R][4]) {
                const unsigned char *row = btl + o * row_stride32(NP) + 16 * h;
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int c = 8 * r + 2 * q + h;  // float4 chunk of states 32 r + 8 q + 4 h
                        b[r][q] = BLDS ? *(const float4 *)(row + 16 * (8 * r + 2 * q))
                                       : ((const float4 *)btk)[(size_t)o * (NP / 4) + c];
                    }
            };

            float acur[R][16];
            int E = 0, E_end = 0;
            float c_end = 1.0f;
            if (Tmax > 0) {
                load_chunk(0);
                store_chunk(0);
                load_chunk(CH32);
                // one step: bcur holds the emission row of step t, bnext receives the
                // one of step t + 1, whose symbol o1 was read from LDS a step earlier,
                // and o2 receives the symbol of step t + 2 (the loops below alternate
                // the buffers, so no copy is needed between steps); cap: whether a
                // sequence of the tile may end at this step (then its sum is kept).  A
                // chunk enters LDS at the step that reads its first symbol, after the
                // last read of the chunk before.
                auto step = [&](auto cap, int t, const float4 (&bcur)[R][4], float4 (&bnext)[R][4], int o1, int &o2,
                                bool full) {
                    const int tn = t + 1;
                    if (tn < Tmax) {
                        gather(o1, bnext);
                        if (tn + 1 < Tmax) {
                            if (((tn + 1) % CH32) == 0) {
                                store_chunk(tn + 1);
                                load_chunk(tn + 1 + CH32);
                            }
                            o2 = read_sym(tn + 1);
                        }
                    }
                    float x[R][16];
                    float part;
                    {
#pragma clang fp contract(off)
                        if (t == 0) {
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int v = 0; v < 16; ++v) {
                                    const int i = 32 * r + 8 * (v / 4) + 4 * h + v % 4;
                                    x[r][v] = (i < N ? pik[i] : 0.0f) * bcur[r][v / 4][v % 4];
                                }
                        } else {
                            // Raised wave priority while the MFMA chain issues, so that a
                            // wave entering its chain is not held behind another wave's
                            // epilogue arithmetic.
                            __builtin_amdgcn_s_setprio(1);
                            floatx16 acc[R];
#pragma unroll
                            for (int r = 0; r < R; ++r) acc[r] = floatx16{};
#pragma unroll
                            for (int rp = 0; rp < R; ++rp)
#pragma unroll
                                for (int v = 0; v < 16; ++v)
#pragma unroll
                                    for (int r = 0; r < R; ++r)
                                        acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[r][rp][v], acur[rp][v], acc[r],
                                                                                      0, 0, 0);
                            __builtin_amdgcn_s_setprio(0);
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int v = 0; v < 16; ++v) x[r][v] = acc[r][v] * bcur[r][v / 4][v % 4];
                        }
                        if (!full) {
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int v = 0; v < 16; ++v) acur[r][v] = x[r][v];
                            return;
                        }
                        part = x[0][0];
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int v = (r == 0 ? 1 : 0); v < 16; ++v) part = part + x[r][v];
                    }
                    auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(part), __float_as_uint(part), false, false);
                    const float cs = __uint_as_float(q[0]) + __uint_as_float(q[1]);
                    const int e = frexp_exp(cs);
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int v = 0; v < 16; ++v) acur[r][v] = ldexp_f(x[r][v], -e);
                    if constexpr (decltype(cap)::value) {
                        if (t == T - 1) {
                            E_end = E;
                            c_end = cs;
                        }
                    }
                    E += e;
                };
                float4 bA[R][4], bB[R][4];
                gather(read_sym(0), bA);
                int oA = 0, oB = read_sym(1);  // symbols of the next even and odd steps
                // steps before Tmin - 1, where no sequence of the tile ends, then the
                // rest, where the sums of ending sequences are kept (the same steps
                // rescale in both loops: every odd one, and every step from Tmin - 1 on
                // or without the lazy rule)
                int t = 0;
                for (; t + 2 < Tmin; t += 2) {
                    step(std::false_type{}, t, bA, bB, oB, oA, !lazy);
                    step(std::false_type{}, t + 1, bB, bA, oA, oB, true);
                }
                for (; t < Tmax; t += 2) {
                    step(std::true_type{}, t, bA, bB, oB, oA, !lazy || t + 1 >= Tmin);
                    if (t + 1 < Tmax) step(std::true_type{}, t + 1, bB, bA, oA, oB, true);
                }
            }
            int sb = symbad ? 1 : 0;
            sb |= __shfl_xor(sb, 32, WAVE);
            if (has && h == 0) {
                float r = (float)((double)E_end * LN2 + (double)logf(c_end));
                if (bad || sb) r = NAN;
                store_ll(f, seq, pos, k, r);
                if (bad || sb) atomicMin(f.err, seq);
            }
        }
    }
}

template <int R, bool BLDS>
hipError_t launch_t(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st) {
    const size_t lds = BLDS ? (size_t)f.M * row_stride32(32 * R) : 0;
    auto kern = k_fwd_mfma32<R, BLDS>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVES32 * WAVE, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const int grid = persistent_grid(cu_count * per_cu, tile_bound(f.S, f.K, f.all_pairs, T32), WAVES32, f.K, f.max_grid);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVES32 * WAVE), lds, st, d, f);
    return hipGetLastError();
}

}  // namespace

bool fwd_mfma32_supported(int NP) { return NP == 32 || NP == 64; }

hipError_t launch_fwd_mfma32(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st) {
    if (f.ckpt != nullptr) return hipErrorInvalidValue;
    const bool blds = bt_in_lds(f);
    switch (f.NP) {
        case 32: return blds ? launch_t<1, true>(d, f, cu_count, st) : launch_t<1, false>(d, f, cu_count, st);
        case 64: return blds ? launch_t<2, true>(d, f, cu_count, st) : launch_t<2, false>(d, f, cu_count, st);
        default: return hipErrorInvalidValue;
    }
}

HMM_DEBUG_TAKE(debug_take_fwd_mfma32)

}  // namespace hmm
