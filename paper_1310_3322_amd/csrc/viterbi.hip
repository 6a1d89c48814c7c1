// Viterbi decoding (gfx950): the most likely hidden state path of each
// sequence under its own model (paper Sec. 2.7, the "Viterbi" function of the
// HMM stage), in the log domain:
//   delta_1(i) = ln pi[i] + ln B[i][o_1]
//   delta_t(j) = max_i (delta_{t-1}(i) + ln A[i][j]) + ln B[j][o_t],   psi_t(j) = first i attaining it
//   score = max_j delta_T(j),  q_T = first j attaining it,  q_{t-1} = psi_t(q_t).
//
// The step is a max-plus product, which the matrix cores do not execute, so it
// runs on the vector ALUs.  Up to 64 states a wave holds 64 / NP length-sorted
// sequences of one model (larger banks: the workgroup decoder further down);
// lane (slot, j) owns state j of its sequence and keeps the column
// ln A[:, j] in registers.  Per step every lane publishes delta_{t-1}(j) in
// LDS, reads the NP values of its sequence (four per read) and forms the
// maximum of the NP candidates (an add and half a three-way maximum each),
// then adds ln B[j][o_t] from the log-emission table ln B^T [K][M][NP].  Every
// RN steps the scores of a sequence are shifted by their maximum (a common
// shift changes no arg-max) and the shifts add up in FP64, which keeps the FP32
// values small and the score accurate to a few ulps of its magnitude.
//
// The decoder stores each step's delta row (the exact FP32 values the next
// step reads) in a [sum T][NP] array laid out like the symbols, instead of an
// arg-max per state: the arg-max is needed for one state per step only, the one
// on the path, so the traceback recomputes it there from the same stored
// operands with the same FP32 additions and takes the first lane attaining the
// maximum.  psi_t(q_t) is therefore exactly the decoder's choice, and the
// decoder does about a third of the vector work of tracking NP arg-maxes.
//
// Bounded storage.  A sequence's rows are needed until its traceback, so
// keeping every row would take sum T x NP floats (36 GB for 16k sequences of
// up to 4096 steps at 256 states).  The work list (every sequence, longest
// first, whatever its model) is instead cut into rounds of consecutive entries
// whose rows fit the workspace; a round is one decoder launch and one
// traceback launch over its entries, and the next round reuses the rows.  An
// entry's rows start at the exclusive prefix of the lengths before it in the
// list (a scan before the first round).  A one-wave launch before each round
// finds its end: the furthest entry whose rows still fit, rounded down to a
// whole number of generations (the sequences the persistent decoder holds at
// once) when at least one generation fits and entries remain, so that a
// round's entries, of nearly equal length, keep every decoder busy until the
// round ends.  With room for every row there is one round.  Lanes take the
// model of their own sequence (ln A from the transposed log table, ln B from
// the emission table of that model), so one unit may mix models.
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

// Order-preserving integer key of a float (no NaN): negative values have
// their magnitude bits flipped, so signed comparison of keys is float
// comparison, and equal keys are equal floats (-0 aside, which the recursion
// never produces: it adds logarithms and subtracts a maximum from itself).
__device__ __forceinline__ int order_key(float x) {
    const int b = __float_as_int(x);
    return b ^ ((b >> 31) & 0x7fffffff);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

// Maximum of the keys over the NP lanes of a group (NP = 16, 32, 64), in every
// lane of the group: row permutations (DPP: swap neighbours, swap pairs,
// mirror the half-row, mirror the row; each fused into one max instruction)
// and the row and half-wave swaps of gfx950, so that no level goes through the
// LDS crossbar.  A maximum is exact in any order.
template <int NP>
__device__ __forceinline__ int group_max_key(int k) {
    k = max(k, dpp_i<0xB1>(k));   // quad_perm [1, 0, 3, 2]
    k = max(k, dpp_i<0x4E>(k));   // quad_perm [2, 3, 0, 1]
    k = max(k, dpp_i<0x141>(k));  // row_half_mirror
    k = max(k, dpp_i<0x140>(k));  // row_mirror
    if constexpr (NP >= 32) {
        auto p = __builtin_amdgcn_permlane16_swap(k, k, false, false);
        k = max((int)p[0], (int)p[1]);
    }
    if constexpr (NP >= 64) {
        auto p = __builtin_amdgcn_permlane32_swap(k, k, false, false);
        k = max((int)p[0], (int)p[1]);
    }
    return k;
}

// Round bookkeeping, in the int32 words of v.state:
//   [0] decoder head, [1] traceback head,
//   [2] start, [3] end, [4] half of the round being decoded,
//   [5] start, [6] end, [7] half of the round before it (being traced),
//   [8] rounds set up so far.
// Entry p of a round stores its rows from row rowpos[p] + roff of the delta
// array, roff = (half ? half_rows : 0) - rowpos[start].
struct VRound {
    int start, end;
    int64_t roff;
};

__device__ __forceinline__ VRound vround(const VitLaunch &v, int at) {
    VRound r;
    r.start = v.state[at];
    r.end = v.state[at + 1];
    r.roff = r.end > r.start ? (v.state[at + 2] ? v.half_rows : 0) - v.rowpos[r.start] : 0;
    return r;
}

// One wave, before each pass: the round decoded so far becomes the one to
// trace, and the next round is [start, end) with start = the previous end and
// end the furthest entry e with rowpos[e] - rowpos[start] <= the round's rows
// (64 probes per level; an entry stores at most that many rows, so e >
// start), rounded down to a multiple of `gen` entries when that keeps at
// least one and entries remain.  With room for every row (half_rows = 0) the
// first round takes every entry into the whole array; otherwise rounds
// alternate between the two halves, so that a round is decoded while the one
// before it is traced.
__global__ void __launch_bounds__(WAVE) k_vit_round(VitLaunch v, int gen) {
    const int lane = threadIdx.x;
    const int S = v.S;
    const int r = v.state[8];
    const int pstart = v.state[2], pend = v.state[3], phalf = v.state[4];
    const int start = pend;
    int end = S;
    if (start < S) {
        const int64_t lim = v.rowpos[start] + (v.half_rows > 0 ? v.half_rows : v.cap_rows);
        if (v.rowpos[S] > lim) {
            int lo = start + 1, hi = S;  // fits at lo, not at hi
            while (hi - lo > 1) {
                const int p = lo + (int)(((int64_t)(hi - lo) * (lane + 1)) / (WAVE + 1));  // lo <= p < hi, nondecreasing
                const bool f = p == lo || v.rowpos[p] <= lim;
                const int nt = __popcll(__ballot(f));  // the probes that fit are lanes 0 .. nt - 1
                const int nlo = nt > 0 ? __shfl(p, nt - 1, WAVE) : lo;
                const int nhi = nt < WAVE ? __shfl(p, nt < WAVE ? nt : 0, WAVE) : hi;
                lo = nlo > lo ? nlo : lo;
                hi = nhi;
            }
            end = lo;
            const int n = end - start;
            if (n >= gen) end = start + n / gen * gen;
        }
        if (!dbg_in(end - start, (int64_t)S - start + 1, HMM_DEBUG_VIT_ROUND)) end = start;
    }
    if (lane == 0) {
        v.state[0] = 0;
        v.state[1] = 0;
        v.state[5] = pstart;
        v.state[6] = pend;
        v.state[7] = phalf;
        v.state[2] = start < S ? start : S;
        v.state[3] = start < S ? end : S;
        v.state[4] = v.half_rows > 0 ? (r & 1) : 0;
        v.state[8] = r + 1;
    }
}

// After the last pass, work-list entries from `from` on were decoded by no
// round (possible only when sequences overlap in the symbol array, so that
// their rows exceed total_symbols): they are reported like invalid ones.
__device__ void mark_unreached(const VitLaunch &v, int from) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < v.S; p += stride) {
        const int s = v.perm[p];
        v.score[s] = NAN;
        atomicMin(v.err, s);
    }
}

// Decoder of one wave over the units of round R; dl: the wave's two LDS
// buffers of WAVE floats.
template <int NP>
__device__ void vit_decode_waves(const DevPtrs &d, const VitLaunch &v, const VRound &R, float *dl) {
    constexpr int SPW = WAVE / NP;  // sequences per wave
    const int lane = threadIdx.x & (WAVE - 1);
    const int slot = lane / NP, j = lane % NP;
    const int K = v.K, N = v.N, M = v.M;
    const int start = R.start, end = R.end;
    const int nunits = (end - start + SPW - 1) / SPW;

    for (;;) {
        const int unit = wave_pop(&v.state[0]);
        if (unit >= nunits) break;

        const int pos = start + unit * SPW + slot;
        const bool has = pos < end;
        const int seq = has ? v.perm[pos] : 0;
        int32_t T = 0;
        int64_t off = 0;
        bool bad = false;
        int k = 0;
        if (has) {
            T = d.lengths[seq];
            off = d.offsets[seq];
            bad = seq_bad(T, off, v.max_len, v.total);
            const int mk = d.model_of_seq[seq];
            bad |= (mk < 0 || mk >= K);
            if (bad) T = 0;
            k = bad ? 0 : mk;
            // the entry's rows lie inside the delta array (debug build: else skipped)
            if (T > 0 && !dbg_in(v.rowpos[pos] + R.roff + T - 1, v.cap_rows, HMM_DEBUG_VIT_ROWS)) T = 0;
        }
        // column j of ln A of this lane's model (states beyond N are impossible)
        float la[NP];
        {
            const float4 *col = (const float4 *)(v.lnat + ((size_t)k * N + (j < N ? j : 0)) * NP);
#pragma unroll
            for (int i4 = 0; i4 < NP / 4; ++i4) {
                const float4 x = col[i4];
                la[4 * i4] = j < N ? x.x : -INFINITY;
                la[4 * i4 + 1] = j < N ? x.y : -INFINITY;
                la[4 * i4 + 2] = j < N ? x.z : -INFINITY;
                la[4 * i4 + 3] = j < N ? x.w : -INFINITY;
            }
        }
        const float lpi = j < N ? logf(d.pi[(size_t)k * N + j]) : -INFINITY;
        const float *lbk = v.lnbt + (size_t)k * M * NP;
        const int Tmax = __builtin_amdgcn_readfirstlane(wave_max_int(T));
        const int32_t *sq = T > 0 ? d.symbols + off : d.symbols;
        const int tlim = T > 0 ? T - 1 : 0;
        // delta_t goes to row min(t, T - 1) of the sequence: the store is unconditional
        // (a store under a lane-dependent branch makes the compiler wait for every
        // outstanding memory operation at the next step), finished lanes rewrite
        // their last row, which the traceback never reads, and empty slots write
        // to a spare area
        float *drow = T > 0 ? v.delta + (size_t)(v.rowpos[pos] + R.roff) * NP + j : v.spill + lane;
        const int rmax = T > 0 ? T - 1 : 0;
        const size_t rstride = T > 0 ? NP : 0;
        bool symbad = false;
        double shift = 0.0;
        float del = -INFINITY;
        float fin_v = -INFINITY;
        int fin_i = 0;
        double fin_shift = 0.0;
        // Software pipeline without loop-carried copies (a copy of a loaded
        // register waits for every outstanding load and store of the wave): the
        // step loop is unrolled by U; ring[u] holds the symbol of step t0 + u and is
        // reloaded with the symbol of step t0 + U + u once read, so that symbols
        // arrive U - 1 steps ahead; the emission term of step t + 1 is requested in
        // step t into the register of the other parity.  Steps past Tmax (at most
        // U - 1 per unit) change nothing that is read: their delta stores go to the
        // last row, their shift and final-state updates are never taken.  A symbol
        // is checked where it is used, one step before its own step.
        constexpr int U = 8;
        auto checked = [&](int o, int t) {
            symbad |= (t < T) && (o < 0 || o >= M);
            return ((unsigned)o < (unsigned)M) ? o : 0;
        };
        int ring[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ring[u] = Tmax > 0 ? sq[min(u, tlim)] : 0;
        float lbv[2];
        lbv[0] = lbk[(size_t)checked(ring[0], 0) * NP + j];
        lbv[1] = 0.0f;
        for (int t0 = 0; t0 < Tmax; t0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u;
                const float lb = lbv[u & 1];
                const int on = ring[(u + 1) % U];  // symbol of step t + 1 (for u = U - 1: reloaded in step 0)
                lbv[(u + 1) & 1] = lbk[(size_t)checked(on, t + 1) * NP + j];
                ring[u] = sq[min(t + U, tlim)];
                if (t == 0) {
                    del = lpi + lb;
                } else {
                    float *buf = dl + (u & 1) * WAVE;
                    buf[lane] = del;
                    wave_lds_sync();
                    const float4 *rw = (const float4 *)(buf + slot * NP);
                    float best = -INFINITY;
#pragma unroll
                    for (int i4 = 0; i4 < NP / 4; ++i4) {
                        const float4 q = rw[i4];
                        best = fmaxf(fmaxf(best, q.x + la[4 * i4]), q.y + la[4 * i4 + 1]);
                        best = fmaxf(fmaxf(best, q.z + la[4 * i4 + 2]), q.w + la[4 * i4 + 3]);
                    }
                    del = best + lb;
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
                // delta_t as step t + 1 reads it (after any shift)
                drow[(size_t)min(t, rmax) * rstride] = del;
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

// Traceback: from q_T (left in path by the decoder) down to q_1.  Each wave
// pops units of 64 / NP entries of the round.  Per step, lane (slot, i) of a
// sequence forms the candidate delta_{t-1}(i) + ln A_k[i][q_t] from the
// stored delta row and row q_t of the transposed log table of its model, the
// group takes the maximum, and the first lane whose candidate equals it gives
// q_{t-1}.  Up to 32 states the wave first copies the tables of its unit's
// models into its LDS area lt (the row for q_t then comes from LDS, not from
// the cache hierarchy); at 64 states it reads them from global memory.  The
// delta rows do not depend on the path, so each lane keeps the rows of the
// next NP steps in flight.  Sequences with an invalid symbol or model get -1
// everywhere (their range is written only when it is valid).
template <int NP>
constexpr int vstage() { return NP <= 32 ? WAVE * NP : 0; }  // floats of a wave's table area

template <int NP>
__device__ void vit_trace_waves(const DevPtrs &d, const VitLaunch &v, const VRound &R, float *lt) {
    constexpr int SPW = WAVE / NP;
    constexpr bool STAGE = vstage<NP>() > 0;
    const int lane = threadIdx.x & (WAVE - 1);
    const int slot = lane / NP, i = lane % NP;
    const int K = v.K, N = v.N;
    const int start = R.start, end = R.end;
    const int nunits = (end - start + SPW - 1) / SPW;

    for (;;) {
        const int unit = wave_pop(&v.state[1]);
        if (unit >= nunits) break;
        const int pos = start + unit * SPW + slot;
        const bool has = pos < end;
        const int s = has ? v.perm[pos] : 0;
        int32_t T = 0;
        int64_t off = 0;
        int k = 0;
        if (has) {
            T = d.lengths[s];
            off = d.offsets[s];
            const int mk = d.model_of_seq[s];
            if (seq_bad(T, off, v.max_len, v.total) || mk < 0 || mk >= K) T = 0;
            else k = mk;
            if (T > 0 && !dbg_in(v.rowpos[pos] + R.roff + T - 1, v.cap_rows, HMM_DEBUG_VIT_ROWS)) T = 0;
        }
        int32_t *q = v.path + (T > 0 ? off : 0);
        const float sc = T > 0 ? v.score[s] : 0.0f;
        if (sc != sc) {  // invalid symbol: no path
            for (int32_t t = i; t < T; t += NP) q[t] = -1;
            T = 0;
        }
        const int Tmax = __builtin_amdgcn_readfirstlane(wave_max_int(T));
        if (Tmax <= 1) continue;
        int cur = T > 0 ? q[T - 1] : 0;
        cur = ((unsigned)cur < (unsigned)N) ? cur : 0;
        // row q of lnt is row q of ln A_k transposed, this lane's entry (q < N)
        const float *lnt;
        if constexpr (STAGE) {
            // slot g's table at lt + g NP^2; every lane copies NP / 4 float4 of them
#pragma unroll 1
            for (int e4 = lane; e4 < SPW * NP * NP / 4; e4 += WAVE) {
                const int e = 4 * e4;
                const int g = e / (NP * NP), q = (e / NP) % NP, ii = e % NP;
                const int kg = __shfl(k, g * NP, WAVE);
                float4 x = make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
                if (q < N) x = *(const float4 *)(v.lnat + ((size_t)kg * N + q) * NP + ii);
                *(float4 *)(lt + e) = x;
            }
            wave_lds_sync();
            lnt = lt + slot * NP * NP + i;
        } else {
            lnt = v.lnat + (size_t)k * N * NP + i;
        }
        // row r (0 <= r <= T - 2) of this lane's sequence holds delta_r(i).  Loads and
        // stores are unconditional (rows clamped into the sequence, stores outside the
        // chunk to a spare area), since a memory operation under a lane-dependent branch
        // makes the compiler wait for every outstanding one at the next step
        const float *drow = T > 1 ? v.delta + (size_t)(v.rowpos[pos] + R.roff) * NP + i : v.spill + lane;
        const int rmax = T > 1 ? T - 2 : 0;
        auto row = [&](int r) { return drow[(uint32_t)min(max(r, 0), rmax) * NP]; };
        int32_t *sink = (int32_t *)v.spill + lane;
        // Blocks of NP wave steps t = t0, t0 - 1, .., t0 - NP + 1, fully unrolled with no
        // exit inside (steps below 1 are dead), so that the ring of delta rows (row t - 1
        // for step t, refilled with the row NP steps further) stays in registers.  Lane i
        // records the state q_{t0 - 1 - i} and the block ends with one coalesced store.
        float ring[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) ring[u] = row(Tmax - 2 - u);
        for (int t0 = Tmax - 1; t0 >= 1; t0 -= NP) {
            int mine = 0;
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const int t = t0 - u;
                const float dprev = ring[u];
                ring[u] = row(t - 1 - NP);
                const bool live = t >= 1 && t < T;
                const int kc = order_key(dprev + lnt[(size_t)cur * NP]);
                // first lane of each group whose candidate is the group's maximum
                const uint64_t hit = __ballot(kc == group_max_key<NP>(kc));
                int nq = 0;
#pragma unroll
                for (int gq = 0; gq < SPW; ++gq) {
                    const uint64_t bg = NP < 64 ? ((hit >> (gq * NP)) | (1ull << (NP & 63))) : hit;
                    const int qg = bg ? (int)__builtin_ctzll(bg) : 0;
                    nq = (gq == 0 || slot == gq) ? qg : nq;
                }
                if (live) cur = nq < N ? nq : 0;
                if (i == u) mine = cur;
            }
            const int st = t0 - 1 - i;
            *((st >= 0 && st <= T - 2) ? q + st : sink) = mine;
        }
    }
}

// Decoder for 64 < N <= 256 (NP = 128 or 256), where a column of ln A no
// longer fits one lane: one sequence per workgroup of 4 NP threads.  The 16
// lanes of a DPP row share a group of WJ = 4 consecutive states j = 4 g + c;
// lane r of the row holds the slice i = r NP / 16 .. (r + 1) NP / 16 - 1 of
// the predecessors, with ln A[i][j] for its slice and the group's 4 states in
// registers (NP / 4 values).  Per step it reads its slice of delta_{t-1} from
// LDS once for the 4 states (four times fewer LDS reads than one state per
// thread), forms the 4 maxima over its slice of delta_{t-1}(i) + ln A[i][j],
// and the row combines them with row-local permutations fused into max
// instructions; lane r then finishes state 4 g + (r & 3) with ln B[j][o_t].
// Recursion, shift period and stored rows are those of the per-wave decoder;
// the maximum for a shift and the final arg-max go through the waves' partial
// results in LDS.  ln A is read from the transposed log table lnat[k][j][i]
// that the traceback reads too, so both form the candidates from identical
// FP32 operands.
constexpr int WJ = 4;     // states per row of 16 lanes
constexpr int WR = 16;    // predecessor slices (the lanes of a row)
constexpr int WSCH = 64;  // symbols per staged chunk

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Maximum over the 16 lanes of a row, in every lane of the row (exact in any order).
__device__ __forceinline__ float row_max(float v) {
    v = fmaxf(v, dpp_f<0xB1>(v));   // quad_perm [1, 0, 3, 2]
    v = fmaxf(v, dpp_f<0x4E>(v));   // quad_perm [2, 3, 0, 1]
    v = fmaxf(v, dpp_f<0x141>(v));  // row_half_mirror
    return fmaxf(v, dpp_f<0x140>(v));  // row_mirror
}

template <int NP>
__device__ void vit_decode_wg(const DevPtrs &d, const VitLaunch &v, const VRound &R) {
    constexpr int IS = NP / WR;                // predecessors per lane
    constexpr int NWV = WR * NP / WJ / WAVE;   // waves per workgroup
    constexpr int SLP = IS + 4;                // padded slice: the 16 slices start on different banks
    __shared__ __align__(16) float dl[2][WR * SLP];
    __shared__ int32_t syms[2][WSCH];
    __shared__ float red_v[NWV];
    __shared__ int red_i[NWV];
    __shared__ int unit_sh;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int jg = tid / WR, r = tid % WR;
    const int j = WJ * jg + (r & (WJ - 1));  // the state this lane finishes
    const int K = v.K, N = v.N, M = v.M;

    const int start = R.start, end = R.end;
    const int nseq = end - start;

    // The loop's exit and the step loop's bound are scalar (readfirstlane): a
    // bound the compiler takes for a per-lane value turns these loops, which
    // contain barriers, into exec-masked loops, and with the pop and the output
    // both under tid == 0 it then let lanes 1..63 of wave 0 re-enter the
    // sequence loop without lane 0, re-reading a head that never advanced.
    for (;;) {
        if (tid == 0) unit_sh = atomicAdd(&v.state[0], 1);
        __syncthreads();
        const int unit = __builtin_amdgcn_readfirstlane(unit_sh);
        __syncthreads();
        if (unit >= nseq) break;

        const int pos = start + unit;
        const int seq = v.perm[pos];
        const int32_t Tin = d.lengths[seq];
        const int64_t off = d.offsets[seq];
        const int mk = d.model_of_seq[seq];
        const bool bad = seq_bad(Tin, off, v.max_len, v.total) || mk < 0 || mk >= K;
        const bool rows_ok = bad || Tin == 0 || dbg_in(v.rowpos[pos] + R.roff + Tin - 1, v.cap_rows, HMM_DEBUG_VIT_ROWS);
        const int32_t T = __builtin_amdgcn_readfirstlane((bad || !rows_ok) ? 0 : Tin);
        const int k = __builtin_amdgcn_readfirstlane(bad ? 0 : mk);
        // ln A[i][4 jg + c] for this lane's slice of i (states beyond N are impossible)
        float la[WJ][IS];
#pragma unroll
        for (int c = 0; c < WJ; ++c) {
            const int jc = WJ * jg + c;
            const float4 *row = (const float4 *)(v.lnat + ((size_t)k * N + (jc < N ? jc : 0)) * NP + r * IS);
#pragma unroll
            for (int i4 = 0; i4 < IS / 4; ++i4) {
                const float4 x = row[i4];
                la[c][4 * i4] = jc < N ? x.x : -INFINITY;
                la[c][4 * i4 + 1] = jc < N ? x.y : -INFINITY;
                la[c][4 * i4 + 2] = jc < N ? x.z : -INFINITY;
                la[c][4 * i4 + 3] = jc < N ? x.w : -INFINITY;
            }
        }
        const float lpi = j < N ? logf(d.pi[(size_t)k * N + j]) : -INFINITY;
        const float *lbk = v.lnbt + (size_t)k * M * NP;
        const int32_t *sq = T > 0 ? d.symbols + off : d.symbols;
        const int tlim = T > 0 ? T - 1 : 0;
        // row t of the sequence's delta rows (the values step t + 1 reads); the
        // lanes that finish the same state store the same value
        float *drow = v.delta + (T > 0 ? (size_t)(v.rowpos[pos] + R.roff) : 0) * NP + j;
        bool symbad = false;
        double shift = 0.0;
        float del = -INFINITY;
        float fin_v = -INFINITY;
        double fin_shift = 0.0;
        if (T > 0) {
            if (tid < WSCH) {
                syms[0][tid] = sq[min(tid, tlim)];
                syms[1][tid] = sq[min(WSCH + tid, tlim)];
            }
            __syncthreads();
            // the symbol of step t (< T), checked once, from the staged chunks
            auto sym_at = [&](int t) {
                const int o = syms[(t / WSCH) & 1][t % WSCH];
                symbad |= (o < 0 || o >= M);
                return ((unsigned)o < (unsigned)M) ? o : 0;
            };
            auto step = [&](int t, float lb) {
                if (t >= WSCH && (t % WSCH) == 0 && tid < WSCH) {
                    // chunk t / WSCH + 1 into the buffer of chunk t / WSCH - 1, whose last
                    // symbol was read before step t - 2; read from step t + WSCH - 1 on
                    syms[((t / WSCH) + 1) & 1][tid] = sq[min(t + WSCH + tid, tlim)];
                }
                if (t == 0) {
                    del = lpi + lb;
                } else {
                    const float4 *pr = (const float4 *)(dl[(t - 1) & 1] + r * SLP);
                    float best[WJ];
#pragma unroll
                    for (int c = 0; c < WJ; ++c) best[c] = -INFINITY;
#pragma unroll
                    for (int i4 = 0; i4 < IS / 4; ++i4) {
                        const float4 x = pr[i4];
#pragma unroll
                        for (int c = 0; c < WJ; ++c) {
                            best[c] = fmaxf(fmaxf(best[c], x.x + la[c][4 * i4]), x.y + la[c][4 * i4 + 1]);
                            best[c] = fmaxf(fmaxf(best[c], x.z + la[c][4 * i4 + 2]), x.w + la[c][4 * i4 + 3]);
                        }
                    }
#pragma unroll
                    for (int c = 0; c < WJ; ++c) best[c] = row_max(best[c]);
                    const int cs = r & (WJ - 1);
                    const float bs = cs == 0 ? best[0] : cs == 1 ? best[1] : cs == 2 ? best[2] : best[3];
                    del = bs + lb;
                }
                if (t == T - 1) {
                    fin_v = del;
                    fin_shift = shift;
                }
                if (((t + 1) % RN) == 0) {
                    float m = group_max<WAVE>(del);
                    if (lane == 0) red_v[wave] = m;
                    __syncthreads();
                    m = red_v[0];
#pragma unroll
                    for (int w2 = 1; w2 < NWV; ++w2) m = fmaxf(m, red_v[w2]);
                    if (!(m > -INFINITY && m < INFINITY)) m = 0.0f;
                    del = del - m;
                    shift += (double)m;
                }
                dl[t & 1][j + (j / IS) * (SLP - IS)] = del;
                drow[(size_t)t * NP] = del;
                lds_barrier();
            };
            // The emission term of a step is requested one step ahead (its
            // gather from the emission table, which the models of a round share
            // in the cache, then overlaps a step of work), in two registers
            // that alternate so that no loaded value is copied.
            float lb0 = lbk[(size_t)sym_at(0) * NP + j], lb1 = 0.0f;
            for (int t = 0; t < T; t += 2) {
                if (t + 1 < T) lb1 = lbk[(size_t)sym_at(t + 1) * NP + j];
                step(t, lb0);
                if (t + 1 < T) {
                    if (t + 2 < T) lb0 = lbk[(size_t)sym_at(t + 2) * NP + j];
                    step(t + 1, lb1);
                }
            }
        }
        // last state: the first state attaining the maximum of delta_T
        float fv = fin_v;
        int fi = j;
        group_argmax<WAVE>(fv, fi);
        if (lane == 0) {
            red_v[wave] = fv;
            red_i[wave] = fi;
        }
        __syncthreads();
        if (tid == 0) {
            float bv = red_v[0];
            int bi = red_i[0];
            for (int w2 = 1; w2 < NWV; ++w2)  // waves hold increasing states
                if (red_v[w2] > bv) {
                    bv = red_v[w2];
                    bi = red_i[w2];
                }
            float sc;
            if (bad || symbad) {
                sc = NAN;
                atomicMin(v.err, seq);
            } else if (T == 0) {
                sc = 0.0f;
            } else {
                sc = (float)(fin_shift + (double)bv);
            }
            v.score[seq] = sc;
            if (T > 0) v.path[off + T - 1] = (bad || symbad) ? -1 : bi;
        }
        __syncthreads();  // the outputs of tid 0 stay apart from its next pop
    }
}

// Traceback for 64 < N <= 256: one wave per sequence, lane l holding the
// predecessors i = 64 c + l (c < NP / 64).  Per step the candidates
// delta_{t-1}(i) + ln A[i][q_t] come from the stored row and the row q_t of
// the transposed log table; the first state attaining their maximum is
// q_{t-1}.  Rows are requested TU steps ahead (they do not depend on the
// path); lane u of a block of TU steps records q_{t0 - 1 - u}, and the block
// ends with one store.
constexpr int TU = 8;

template <int NP>
__device__ void vit_trace_wave_wg(const DevPtrs &d, const VitLaunch &v, const VRound &R) {
    constexpr int C = NP / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int K = v.K, N = v.N;
    const int start = R.start, end = R.end;
    const int nseq = end - start;

    for (;;) {
        const int unit = wave_pop(&v.state[1]);
        if (unit >= nseq) break;
        const int pos = start + unit;
        const int s = v.perm[pos];
        int32_t T = d.lengths[s];
        const int64_t off = d.offsets[s];
        const int mk = d.model_of_seq[s];
        const bool bad = seq_bad(T, off, v.max_len, v.total) || mk < 0 || mk >= K;
        if (bad) T = 0;
        if (T > 0 && !dbg_in(v.rowpos[pos] + R.roff + T - 1, v.cap_rows, HMM_DEBUG_VIT_ROWS)) T = 0;
        const int k = __builtin_amdgcn_readfirstlane(bad ? 0 : mk);
        const float *lnk = v.lnat + (size_t)k * N * NP;
        int32_t *qp = v.path + (T > 0 ? off : 0);
        const float sc = T > 0 ? v.score[s] : 0.0f;
        if (sc != sc) {  // invalid symbol: no path
            for (int32_t t = lane; t < T; t += WAVE) qp[t] = -1;
            T = 0;
        }
        T = __builtin_amdgcn_readfirstlane(T);  // one sequence per wave: scalar loop bounds
        if (T <= 1) continue;
        int cur = __builtin_amdgcn_readfirstlane(qp[T - 1]);
        cur = ((unsigned)cur < (unsigned)N) ? cur : 0;
        const float *drow = v.delta + (size_t)(v.rowpos[pos] + R.roff) * NP + lane;
        auto row = [&](int r, int c) { return drow[(size_t)max(r, 0) * NP + c * WAVE]; };
        int32_t *sink = (int32_t *)v.spill + lane;
        float ring[TU][C];
#pragma unroll
        for (int u = 0; u < TU; ++u)
#pragma unroll
            for (int c = 0; c < C; ++c) ring[u][c] = row(T - 2 - u, c);
        for (int t0 = T - 1; t0 >= 1; t0 -= TU) {
            int mine = 0;
#pragma unroll
            for (int u = 0; u < TU; ++u) {
                const int t = t0 - u;
                float dprev[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    dprev[c] = ring[u][c];
                    ring[u][c] = row(t - 1 - TU, c);
                }
                const float *lr = lnk + (size_t)cur * NP + lane;
                int kc[C];
                int m = INT_MIN;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    kc[c] = order_key(dprev[c] + lr[c * WAVE]);
                    m = max(m, kc[c]);
                }
                m = group_max_key<WAVE>(m);
                int nq = -1;
#pragma unroll
                for (int c = C - 1; c >= 0; --c) {  // the lowest block with a hit wins
                    const uint64_t h = __ballot(kc[c] == m);
                    if (h) nq = c * WAVE + (int)__builtin_ctzll(h);
                }
                if (t >= 1) cur = (nq >= 0 && nq < N) ? nq : 0;
                if (lane == u) mine = cur;
            }
            const int st = t0 - 1 - lane;
            *((lane < TU && st >= 0) ? qp + st : sink) = mine;
        }
    }
}

// One pass: decode the round set up last and trace back the one before it
// (rows in the other half), in one persistent launch.  The first `tracers`
// waves (workgroups for the workgroup decoder) trace first and decode only
// when there is nothing to trace; the others decode first and then help with
// what is left to trace.  So the traceback of a round, a dependent chain per
// sequence that leaves most of the chip idle on its own, runs beside the next
// round's decoding on a few reserved waves.  In the last pass nothing is
// decoded.
template <int NP>
__global__ void __launch_bounds__(VWAVES * WAVE) k_vit_pass(DevPtrs d, VitLaunch v, int tracers, int last) {
    constexpr int AREA = 2 * WAVE + vstage<NP>();
    __shared__ __align__(16) float lds[VWAVES * AREA];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    float *dl = lds + wave * AREA;
    float *lt = dl + 2 * WAVE;
    const VRound cur = vround(v, 2), prev = vround(v, 5);
    if (last) mark_unreached(v, cur.start);
    const bool dec = !last && cur.end > cur.start;
    const bool trc = prev.end > prev.start;
    if ((int)blockIdx.x * VWAVES + wave < tracers) {
        if (trc) {
            vit_trace_waves<NP>(d, v, prev, lt);
        } else if (dec) {
            vit_decode_waves<NP>(d, v, cur, dl);
        }
    } else {
        if (dec) vit_decode_waves<NP>(d, v, cur, dl);
        if (trc) vit_trace_waves<NP>(d, v, prev, lt);
    }
}

template <int NP>
__global__ void __launch_bounds__(WR * NP / WJ) k_vit_pass_wg(DevPtrs d, VitLaunch v, int tracers, int last) {
    const VRound cur = vround(v, 2), prev = vround(v, 5);
    if (last) mark_unreached(v, cur.start);
    const bool dec = !last && cur.end > cur.start;
    const bool trc = prev.end > prev.start;
    if ((int)blockIdx.x < tracers) {
        if (trc) {
            vit_trace_wave_wg<NP>(d, v, prev);
        } else if (dec) {
            vit_decode_wg<NP>(d, v, cur);
        }
    } else {
        if (dec) vit_decode_wg<NP>(d, v, cur);
        if (trc) vit_trace_wave_wg<NP>(d, v, prev);
    }
}

// The last pass traces the last round only: a kernel of its own, which
// holds fewer registers than the decoder and so more waves per CU (the
// traceback is a dependent chain per sequence).
template <int NP>
__global__ void __launch_bounds__(VWAVES * WAVE) k_vit_trace_pass(DevPtrs d, VitLaunch v) {
    __shared__ __align__(16) float lds[VWAVES * (vstage<NP>() > 0 ? vstage<NP>() : 1)];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const VRound cur = vround(v, 2), prev = vround(v, 5);
    mark_unreached(v, cur.start);
    if (prev.end > prev.start) {
        if constexpr (NP > WAVE)
            vit_trace_wave_wg<NP>(d, v, prev);
        else
            vit_trace_waves<NP>(d, v, prev, lds + wave * vstage<NP>());
    }
}

template <int NP>
hipError_t launch_rounds(const DevPtrs &d, const VitLaunch &v0, int cu_count, hipStream_t st) {
    constexpr bool WG = NP > WAVE;
    constexpr int SPW = WG ? 1 : WAVE / NP;
    constexpr int THREADS = WG ? WR * NP / WJ : VWAVES * WAVE;
    constexpr int UNITS_PER_WG = WG ? 1 : VWAVES;  // decoder units a workgroup holds at once
    const void *kern;
    if constexpr (WG)
        kern = (const void *)k_vit_pass_wg<NP>;
    else
        kern = (const void *)k_vit_pass<NP>;
    int per_cu = 0, per_cu_t = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, THREADS, 0);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_t, (const void *)k_vit_trace_pass<NP>, VWAVES * WAVE, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    if (per_cu_t < 1) per_cu_t = 1;
    const int64_t units = ((int64_t)v0.S + SPW - 1) / SPW;
    const int grid = persistent_grid(cu_count * per_cu, units, UNITS_PER_WG, 1, v0.max_grid);
    const int grid_t = persistent_grid(cu_count * per_cu_t, units, VWAVES, 1, v0.max_grid);
    // tracers: a sixteenth of the decoders (workgroups of the workgroup decoder, waves otherwise)
    const int slots = WG ? grid : grid * VWAVES;
    const int tracers = slots >= 16 ? slots / 16 : 0;
    const int gen = (slots - tracers) * SPW;  // entries the decoders hold at once
    VitLaunch v = v0;
    // rounds in two halves unless every row fits at once
    v.half_rows = v.cap_rows >= v.total ? 0 : v.cap_rows / 2;
    // Each round but the last holds at least one entry, and a whole
    // generation or more or rows beyond half_rows - max_len (the next entry
    // did not fit).  Sequences that do not overlap store at most
    // total_symbols rows, which bounds the rounds.
    int64_t rounds = 1;
    if (v.half_rows > 0) {
        const int64_t per = v.half_rows - v.max_len + 1;
        rounds = (int64_t)v.S / gen + (per > 0 ? v.total / per : v.total);
        if (rounds > v.S - 1) rounds = v.S - 1;
        rounds += 1;
    }
    for (int64_t r = 0; r <= rounds; ++r) {
        hipLaunchKernelGGL(k_vit_round, dim3(1), dim3(WAVE), 0, st, v, gen);
        if (r == rounds)  // the pass after the last round only traces
            hipLaunchKernelGGL(k_vit_trace_pass<NP>, dim3(grid_t), dim3(VWAVES * WAVE), 0, st, d, v);
        else if constexpr (WG)
            hipLaunchKernelGGL(k_vit_pass_wg<NP>, dim3(grid), dim3(THREADS), 0, st, d, v, tracers, 0);
        else
            hipLaunchKernelGGL(k_vit_pass<NP>, dim3(grid), dim3(THREADS), 0, st, d, v, tracers, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

bool viterbi_supported(int NP) { return NP == 16 || NP == 32 || NP == 64 || NP == 128 || NP == 256; }

int64_t viterbi_min_rows(int64_t max_len, int64_t total) {
    // one round with room for every row, or two halves of at least max_len rows
    return total <= 2 * max_len ? total : 2 * max_len;
}

hipError_t launch_viterbi(const DevPtrs &d, const VitLaunch &v, int cu_count, hipStream_t st) {
    if (v.S == 0) return hipSuccess;
    if (!viterbi_supported(v.NP)) return hipErrorInvalidValue;
    if (v.cap_rows < viterbi_min_rows(v.max_len, v.total)) return hipErrorInvalidValue;
    // rows of every entry before it (a decoder row of a sequence with an invalid
    // model is never written, but counting it keeps the sum an upper bound); the
    // round state starts at zero (no round yet)
    const RowPrefix rp{v.perm, v.S, v.max_len, v.total, const_cast<int64_t *>(v.rowpos), v.rowsum, v.state,
                       VIT_STATE_WORDS};
    const hipError_t e = launch_row_prefix(d, rp, st);
    if (e != hipSuccess) return e;
    switch (v.NP) {
        case 16: return launch_rounds<16>(d, v, cu_count, st);
        case 32: return launch_rounds<32>(d, v, cu_count, st);
        case 64: return launch_rounds<64>(d, v, cu_count, st);
        case 128: return launch_rounds<128>(d, v, cu_count, st);
        case 256: return launch_rounds<256>(d, v, cu_count, st);
        default: return hipErrorInvalidValue;
    }
}

HMM_DEBUG_TAKE(debug_take_viterbi)

}  // namespace hmm
