// Batched forward kernel on FP32 MFMA (gfx950): the hot path.
//
// Recognition scores every symbol stream against every activity HMM, and the
// HMMs of the actions are independent (paper Sec. 2.7 and Sec. 3 item 3), so
// for one model k and a tile of 16 length-sorted sequences the forward step
//     u[s][j] = sum_i alphahat_{t-1}[s][i] A_k[i][j]
// is a dense (16 x N) by (N x N) product.  It runs as 16x16x4 FP32 MFMAs in
// the transposed form U^T = A_k^T alphahat^T: the MFMA A operand is A_k^T (kept
// in registers for the whole model), the B operand is alphahat^T, and the
// 16x16 result tile leaves each lane holding one sequence (lane % 16) and four
// consecutive states of each 16-state block (4 * (lane / 16) + 0..3).  The
// contraction order over i is free, so the k-step (block r', register v) feeds
// lane group g the state 16 r' + 4 g + v -- exactly what that lane holds after
// the previous step: the result registers of step t are the B operand of step
// t+1, with no data movement between steps.
//
// Per step and tile (Sec. 2.7 "Forward", renormalised every step):
//   alpha~[s][j] = u[s][j] * B_k[j][o_t(s)]      (row o_t of B^T, from LDS or L2)
//   c_t[s]       = sum_j alpha~[s][j]             (in-lane sum + two row swaps)
//   alphahat     = alpha~ * 2^-e_t, c_t = m_t 2^e_t, m_t in [0.5, 1)  (exact)
//   log P        = (sum_{t<T} e_t) ln 2 + ln c_T  (= sum_t ln c_t)
//
// Work distribution: each workgroup serves one model at a time; its waves pop
// 16-sequence tiles of that model's length-sorted list from a per-model
// queue (longest first), so uneven lengths are balanced inside one launch.
// With K a multiple of 8 all workgroups of a model land on one XCD.
#include <climits>
#include <type_traits>

#include "common.cuh"
#include "fwd_step.cuh"
#include "kernels.h"

namespace hmm {
namespace {

constexpr int CH = 32;               // symbols per staging chunk (multiple of 4)
constexpr int SYM_INTS = CH * TILE;  // one chunk buffer per wave
constexpr int FWD_WAVES = 4;         // waves per workgroup
constexpr size_t LDS_CU = 160 * 1024;

// B^T rows in LDS, row o at byte o * row_stride16(NP): NP floats and 16 bytes of
// padding, an odd number of 16-byte chunks per row, so that chunk c of row o starts
// in bank group (o (NP / 4 + 1) + c) mod 16 and the 16 lanes of one 16-byte LDS
// pass, which read one chunk of 16 random rows, spread over all 16 groups; a lane's
// chunks of a row sit at fixed offsets from one address.
__host__ __device__ constexpr int row_stride16(int NP) { return NP * 4 + 16; }

template <int R, bool BLDS, bool CKPT>
__global__ void __launch_bounds__(FWD_WAVES * WAVE) k_fwd_mfma(DevPtrs d, FwdLaunch f) {
    constexpr int NP = 16 * R;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int sl = lane & 15;        // sequence slot in the tile
    const int g = lane >> 4;         // row group: states 16r + 4g + 0..3
    const int K = f.K, N = f.N, M = f.M;
    unsigned char *btl = smem;       // padded rows of B^T when BLDS
    __shared__ int32_t sym_all[FWD_WAVES * SYM_INTS];   // separate object: never aliases btl
    int32_t *sym = sym_all + wave * SYM_INTS;

    const int G = gridDim.x;
    const int k_first = G >= K ? (int)(blockIdx.x % K) : (int)blockIdx.x;
    const int k_step = G >= K ? K : G;
    for (int k = k_first; k < K; k += k_step) {
        const int grp = f.all_pairs ? 0 : k;
        const int gbeg = f.gstart[grp], gend = f.gstart[grp + 1];
        const int ntiles = (gend - gbeg + TILE - 1) / TILE;
        const float *btk = f.bt + (size_t)k * M * NP;
        if (BLDS) {
            __syncthreads();
            const int n4 = M * NP / 4;
            for (int i = threadIdx.x; i < n4; i += blockDim.x) {
                const int o = i / (NP / 4), c = i % (NP / 4);
                *(float4 *)(btl + o * row_stride16(NP) + 16 * c) = ((const float4 *)btk)[i];
            }
            __syncthreads();
        }
        if (ntiles == 0) continue;
        float af[R][R][4];
        load_fwd_fragments<R>(af, d.A + (size_t)k * N * N, N, g, sl);
        const float *pik = d.pi + (size_t)k * N;

        for (;;) {
            const int tile = wave_pop(&f.queue[k]);
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
            // Shortest sequence of the tile: only its last steps can end a sequence.
            const int Tmin = __builtin_amdgcn_readfirstlane(-wave_max_int(T > 0 ? -T : INT_MIN + 1));
            // Symbols travel in chunks of CH steps: the next chunk is loaded into
            // registers (nxt[u] = symbol of sequence sl at step t0 + (CH / 4) g + u,
            // consecutive, so that a quarter inside the sequence takes 16-byte loads
            // from one address) while the current one is read from the wave's LDS
            // buffer, laid out as sym[u][lane] for the same (u, lane).  Past a
            // sequence's end the loads repeat its last symbol (a valid address;
            // never used).  Symbols are checked and clamped to [0, M) once, when a
            // chunk enters LDS.
            const int32_t *sbase = T > 0 ? d.symbols + off : d.symbols;
            const int tlim = T > 0 ? T - 1 : 0;
            int32_t nxt[CH / 4];
            bool symbad = false;
            auto load_chunk = [&](int t0) {
                const int tb = t0 + (CH / 4) * g;
                if (__builtin_amdgcn_ballot_w64(tb + CH / 4 - 1 > tlim) == 0) {  // every lane's quarter inside
#pragma unroll
                    for (int u = 0; u < CH / 4; u += 4) {
                        int4 v;
                        __builtin_memcpy(&v, sbase + tb + u, 16);  // 4-byte aligned: any global address
                        nxt[u] = v.x;
                        nxt[u + 1] = v.y;
                        nxt[u + 2] = v.z;
                        nxt[u + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < CH / 4; ++u) nxt[u] = sbase[min(tb + u, tlim)];
                }
            };
            auto store_chunk = [&](int t0) {
                wave_lds_sync();
#pragma unroll
                for (int u = 0; u < CH / 4; ++u) {
                    const int o = nxt[u];
                    const bool ok = (unsigned)o < (unsigned)M;
                    symbad |= (t0 + (CH / 4) * g + u < T) && !ok;
                    sym[u * WAVE + lane] = ok ? o : 0;
                }
                wave_lds_sync();
            };
            auto read_sym = [&](int t) {
                const int pp = t % CH;
                return sym[(pp % (CH / 4)) * WAVE + 16 * (pp / (CH / 4)) + sl];
            };
            // chunks 4 r + g of row o of B^T in LDS
            auto gather_lds = [&](int o, float4 (&b)[R]) {
                const unsigned char *row = btl + o * row_stride16(NP) + 16 * g;
#pragma unroll
                for (int r = 0; r < R; ++r) b[r] = *(const float4 *)(row + 64 * r);
            };
            int L = 1, ck_base = 0, ck_t = 0;  // ck_t: next checkpointed step
            if (CKPT) {
                while (L * L < Tmax) ++L;
                ck_base = pos;
            }

            float acur[R][4];
            int E = 0;
            int E_end = 0;        // sum of e_t over t < T - 1 (exponent part of log P)
            float c_end = 1.0f;   // c_T, the last step's sum (log P = E_end ln 2 + ln c_T)
            if (Tmax > 0) {
                load_chunk(0);
                store_chunk(0);
                load_chunk(CH);
                // the emission row of step t + 1 and the symbol of step t + 2 are
                // fetched during step t; a chunk enters LDS at the step that reads its
                // first symbol, after the last read of the chunk before
                float4 b_nx[R];
                {
                    const int o0 = read_sym(0);
                    if (BLDS)
                        gather_lds(o0, b_nx);
                    else
                        gather_b<R>(&btk[(size_t)o0 * NP], g, b_nx);
                }
                int o_nx = read_sym(1);
                // cap: whether a sequence of the tile may end at step t (then its sum
                // is kept); the steps before Tmin - 1 run without that bookkeeping
                auto step = [&](auto cap, int t) {
                    float4 bcur[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) bcur[r] = b_nx[r];
                    const int tn = t + 1;
                    if (tn < Tmax) {
                        if (BLDS)
                            gather_lds(o_nx, b_nx);
                        else
                            gather_b<R>(&btk[(size_t)o_nx * NP], g, b_nx);
                        if (tn + 1 < Tmax) {
                            if (((tn + 1) % CH) == 0) {
                                // chunk (tn + 1) / CH was prefetched a chunk ago
                                store_chunk(tn + 1);
                                load_chunk(tn + 1 + CH);
                            }
                            o_nx = read_sym(tn + 1);
                        }
                    }
                    floatx4 u[R];
                    if (t == 0)
                        pi_as_u<R>(pik, N, g, u);
                    else
                        tile_matvec<R>(af, acur, u);
                    int e;
                    const float cs = emit_and_rescale<R>(u, bcur, acur, e);
                    if constexpr (decltype(cap)::value) {
                        if (t == T - 1) {
                            E_end = E;
                            c_end = cs;
                        }
                    }
                    E += e;
                    if (CKPT && t == ck_t) {  // t = L c
                        const int c = t / L;
                        if (t < T && dbg_in(c, f.nck, HMM_DEBUG_CKPT)) {
                            float *dst = f.ckpt + ((size_t)ck_base * f.nck + c) * NP;
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                *(float4 *)&dst[16 * r + 4 * g] =
                                    float4{acur[r][0], acur[r][1], acur[r][2], acur[r][3]};
                            if (g == 0) f.ckexp[(size_t)ck_base * f.nck + c] = e;
                        }
                        ck_t += L;
                    }
                };
                int t = 0;
                for (; t + 1 < Tmin; ++t) step(std::false_type{}, t);
                for (; t < Tmax; ++t) step(std::true_type{}, t);
            }
            // symbols were checked by the lane that loaded them: combine the four
            // lanes of each sequence
            int sb = symbad ? 1 : 0;
            sb |= __shfl_xor(sb, 16, WAVE);
            sb |= __shfl_xor(sb, 32, WAVE);
            symbad = sb != 0;
            if (has && g == 0) {
                float r = (float)((double)E_end * LN2 + (double)logf(c_end));
                if (bad || symbad) r = NAN;
                store_ll(f, seq, pos, k, r);
                if (bad || symbad) atomicMin(f.err, seq);
                // the backward pass skips sequences without a finite likelihood
                if (CKPT) f.flag[pos] = (r > -INFINITY && r < INFINITY) ? 0 : 1;
            }
        }
    }
}

template <int R, bool BLDS, bool CKPT>
hipError_t launch_t(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st) {
    const size_t lds = BLDS ? (size_t)f.M * row_stride16(16 * R) : 0;  // + static symbol buffers
    auto kern = k_fwd_mfma<R, BLDS, CKPT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, FWD_WAVES * WAVE, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const int grid = persistent_grid(cu_count * per_cu, tile_bound(f.S, f.K, f.all_pairs, TILE), FWD_WAVES, f.K, f.max_grid);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(FWD_WAVES * WAVE), lds, st, d, f);
    return hipGetLastError();
}

}  // namespace

bool fwd_mfma_supported(int NP) { return NP == 16 || NP == 32 || NP == 48 || NP == 64; }

hipError_t launch_fwd_mfma(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st) {
    // the padded rows and the symbol buffers must fit a CU's LDS (the largest table the
    // tuning flag allows, 128 KB, does not with 16 states)
    const bool blds = bt_in_lds(f) && (size_t)f.M * row_stride16(f.NP) + FWD_WAVES * SYM_INTS * sizeof(int32_t) <= LDS_CU;
    const bool ck = f.ckpt != nullptr;
#define HMM_FWD_CASE(R)                                                                  \
    case R:                                                                              \
        if (ck) return blds ? launch_t<R, true, true>(d, f, cu_count, st)                \
                            : launch_t<R, false, true>(d, f, cu_count, st);              \
        return blds ? launch_t<R, true, false>(d, f, cu_count, st)                       \
                    : launch_t<R, false, false>(d, f, cu_count, st);
    switch (f.NP / 16) {
        HMM_FWD_CASE(1)
        HMM_FWD_CASE(2)
        HMM_FWD_CASE(3)
        HMM_FWD_CASE(4)
        default:
            return hipErrorInvalidValue;
    }
#undef HMM_FWD_CASE
}

HMM_DEBUG_TAKE(debug_take_fwd_mfma)

}  // namespace hmm
