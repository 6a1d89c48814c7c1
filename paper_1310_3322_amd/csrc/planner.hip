// Planner and small utility kernels of libhmm_mi355x (gfx950).
//
// The planner turns the ragged batch into one length-sorted work list, the
// batching axis of the paper's independent task parallelism (the HMMs of all
// actions run in parallel, Sec. 3 item 3): a counting sort of the sequence
// ids by (group, descending length), where a group is the owning model when
// each sequence is scored against its own model and the whole batch when every
// sequence is scored against every model.  Tiles of 16 consecutive entries of
// that order then hold sequences of nearly equal length, and the longest tiles
// are handed out first.
#include <climits>
#include <cstring>

#include "common.cuh"
#include "kernels.h"

namespace hmm {
namespace {

// The sort is stable: within a bin, sequences keep their index order, so the
// work list (and with it the composition of every tile) is a function of the
// batch alone.  The batch is cut into chunks of `chunk` consecutive sequences;
// cnt[bin][c] counts the sequences of chunk c in each bin, an exclusive scan of
// cnt in (bin, chunk) order gives every (bin, chunk) its first position, and
// each chunk places its own sequences by their rank among the chunk's
// sequences of the same bin (a sort of (bin, index) keys in LDS).

__global__ void k_plan_init(int32_t *cnt, int64_t n, int32_t *queue, int nq, int32_t *err, uint32_t *bmin, int K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = i; b < n; b += stride) cnt[b] = 0;
    for (int64_t k = i; k < nq; k += stride) queue[k] = 0;
    if (bmin)
        for (int64_t k = i; k < K; k += stride) bmin[k] = 0x7f800000u;
    if (i == 0) *err = INT32_MAX;
}

__device__ __forceinline__ int plan_bin(const DevPtrs &d, int s, int K, int groups, int max_len, int64_t total,
                                        bool *bad_out) {
    int32_t T = d.lengths[s];
    int64_t off = d.offsets[s];
    bool bad = seq_bad(T, off, max_len, total);
    int g = 0;
    if (groups > 1) {
        int mk = d.model_of_seq[s];
        if (mk < 0 || mk >= K) {
            bad = true;
            mk = 0;
        }
        g = mk;
    }
    int te = bad ? 0 : T;
    *bad_out = bad;
    return g * (max_len + 1) + (max_len - te);
}

// One 32 x 32 tile (symbols o0.., states i0.. of model k) of the emission table
// transposed through LDS: dst[k][o][i] = B[k][i][o] for i < N (ln B when `lg`),
// padding 0 (-inf when `lg`) for N <= i < NP; with bmin, bmin[k] takes the bits of
// the smallest B[k][i][o] (non-negative floats order like their bit patterns; bmin
// starts at +inf).  256 threads, tx = t mod 32, ty = t / 32.
__device__ __forceinline__ void transpose_tile(const TransposeJob &j, int k, int o0, int i0, int tx, int ty,
                                               float (*tile)[33], uint32_t *wmin) {
    const int N = j.N, M = j.M, NP = j.NP;
    const float *Bk = j.B + (size_t)k * N * M;
    float *dk = j.dst + (size_t)k * M * NP;
    uint32_t m = 0x7f800000u;
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, o = o0 + tx;
        const bool in = i < N && o < M;
        const float x = in ? Bk[(size_t)i * M + o] : 0.0f;
        tile[r][tx] = j.lg ? (in ? logf(x) : -INFINITY) : x;
        if (in) m = min(m, __float_as_uint(x));
    }
    if (j.bmin) {
        for (int off = 32; off >= 1; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off, WAVE));
        const int t = ty * 32 + tx;
        if ((t & (WAVE - 1)) == 0) wmin[t / WAVE] = m;
    }
    __syncthreads();
    if (j.bmin && tx == 0 && ty == 0) atomicMin(&j.bmin[k], min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3])));
    for (int r = ty; r < 32; r += 8) {
        const int o = o0 + r, i = i0 + tx;
        if (o < M && i < NP) dk[(size_t)o * NP + i] = tile[tx][r];
    }
}

__device__ __forceinline__ void transpose_block(const TransposeJob &j, int blk, int tx, int ty) {
    __shared__ float tile[32][33];
    __shared__ uint32_t wmin[4];
    const int bx = (j.M + 31) / 32, by = (j.NP + 31) / 32;
    const int k = blk / (bx * by), r = blk % (bx * by);
    transpose_tile(j, k, (r % bx) * 32, (r / bx) * 32, tx, ty, tile, wmin);
}

__global__ void __launch_bounds__(256) k_transpose(TransposeJob j) {
    transpose_block(j, blockIdx.x, threadIdx.x & 31, threadIdx.x >> 5);
}

// Blocks below count_blocks count sequences into cnt; the blocks behind them
// transpose the emission table (the two jobs are independent; one launch).
__global__ void __launch_bounds__(256) k_plan_count(DevPtrs d, int S, int K, int groups, int max_len, int64_t total,
                                                    int chunk, int nchunks, int32_t *cnt, int32_t *err,
                                                    int count_blocks, TransposeJob tj) {
    if ((int)blockIdx.x >= count_blocks) {
        transpose_block(tj, blockIdx.x - count_blocks, threadIdx.x & 31, threadIdx.x >> 5);
        return;
    }
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    bool bad;
    const int b = plan_bin(d, s, K, groups, max_len, total, &bad);
    atomicAdd(&cnt[(int64_t)b * nchunks + s / chunk], 1);  // integer: the count is order-independent
    if (bad) atomicMin(err, s);
}

// Exclusive scan of cnt (in place) in (bin, chunk) order, plus the start of
// every group: blocks of PLAN_SCAN entries (8 per thread of 1024); their sums,
// scanned by one workgroup, offset each block's own scan.
constexpr int PLAN_SCAN = 8192;

__global__ void __launch_bounds__(1024) k_plan_scan_reduce(const int32_t *cnt, int64_t n, int32_t *bsum) {
    __shared__ int32_t part[1024];
    const int64_t base = (int64_t)blockIdx.x * PLAN_SCAN;
    int32_t x = 0;
    for (int j = threadIdx.x; j < PLAN_SCAN; j += 1024)
        if (base + j < n) x += cnt[base + j];
    part[threadIdx.x] = x;
    __syncthreads();
    for (int off = 512; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = part[0];
}

// Inclusive scan of 1024 values in LDS (Hillis-Steele); returns the thread's value.
__device__ __forceinline__ int32_t block_inclusive_scan(int32_t *part, int32_t x) {
    const int tid = threadIdx.x;
    part[tid] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    return part[tid];
}

// One workgroup: exclusive scan of the nb block sums in place (pieces of 1024).
__global__ void __launch_bounds__(1024) k_plan_scan_top(int32_t *bsum, int nb) {
    __shared__ int32_t part[1024];
    int32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + (int)threadIdx.x;
        const int32_t x = b < nb ? bsum[b] : 0;
        const int32_t inc = block_inclusive_scan(part, x);
        if (b < nb) bsum[b] = carry + inc - x;
        carry += part[1023];
        __syncthreads();
    }
}

// Small matrices (up to PLAN_SCAN_ONE entries): one workgroup, in one launch.
// The matrix is staged through LDS with coalesced loads and stores (one pad word
// after every 32 entries, so that the threads' runs start on different banks);
// each thread scans a contiguous run of at most 32 entries there.
constexpr int64_t PLAN_SCAN_ONE = 32768;
__host__ __device__ inline int64_t scan_one_pos(int64_t e) { return e + (e >> 5); }
inline size_t scan_one_lds(int64_t n) { return (size_t)(scan_one_pos(n) + 1) * sizeof(int32_t); }

__global__ void __launch_bounds__(1024) k_plan_scan_one(int32_t *cnt, int64_t n, int nchunks, int bins_per_group,
                                                        int groups, int32_t *gstart) {
    __shared__ int32_t part[1024];
    extern __shared__ int32_t stage[];  // entry e at scan_one_pos(e)
    for (int64_t e = threadIdx.x; e < n; e += 1024) stage[scan_one_pos(e)] = cnt[e];
    __syncthreads();
    const int64_t per = (n + 1023) / 1024;
    const int64_t e0 = min(n, (int64_t)threadIdx.x * per), e1 = min(n, e0 + per);
    int32_t local = 0;
    for (int64_t e = e0; e < e1; ++e) local += stage[scan_one_pos(e)];
    int32_t run = block_inclusive_scan(part, local) - local;
    for (int64_t e = e0; e < e1; ++e) {
        const int32_t c = stage[scan_one_pos(e)];
        stage[scan_one_pos(e)] = run;
        const int64_t b = e / nchunks;
        if (e % nchunks == 0 && b % bins_per_group == 0) gstart[b / bins_per_group] = run;
        run += c;
    }
    if (threadIdx.x == 1023) gstart[groups] = part[1023];
    __syncthreads();
    for (int64_t e = threadIdx.x; e < n; e += 1024) cnt[e] = stage[scan_one_pos(e)];
}

__global__ void __launch_bounds__(1024) k_plan_scan_apply(int32_t *cnt, int64_t n, const int32_t *bsum, int nchunks,
                                                          int bins_per_group, int groups, int32_t *gstart) {
    __shared__ int32_t part[1024];
    const int64_t base = (int64_t)blockIdx.x * PLAN_SCAN + (int64_t)threadIdx.x * 8;
    int32_t v[8];
    int32_t local = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = base + j < n ? cnt[base + j] : 0;
        local += v[j];
    }
    int32_t run = bsum[blockIdx.x] + block_inclusive_scan(part, local) - local;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int64_t e = base + j;
        if (e < n) {
            cnt[e] = run;
            const int64_t b = e / nchunks;
            if (e % nchunks == 0 && b % bins_per_group == 0) gstart[b / bins_per_group] = run;
        }
        run += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 1023) gstart[groups] = run;
}

constexpr int PLAN_SUB = 2048;  // keys sorted at a time by a scatter workgroup (11 bits of index)

// One workgroup of 1024 threads per chunk; the chunk's sequences are taken
// PLAN_SUB at a time in index order.  Keys (bin << 11 | index within the
// sub-chunk) are unique, so the sort's result is fixed; a sequence's
// rank within its bin is its sorted position minus the first position of its
// bin (binary search), its place cnt[bin][chunk] + rank.  Between sub-chunks
// the last sequence of each bin advances cnt[bin][chunk].
__global__ void __launch_bounds__(1024) k_plan_scatter(DevPtrs d, int S, int K, int groups, int max_len,
                                                       int64_t total, int chunk, int nchunks, int32_t *cnt,
                                                       int32_t *perm) {
    __shared__ uint64_t key[PLAN_SUB];
    const int tid = threadIdx.x;
    const int c = blockIdx.x;
    const int cbeg = c * chunk, cend = min(S, cbeg + chunk);
    for (int base = cbeg; base < cend; base += PLAN_SUB) {
        const int n = min(PLAN_SUB, cend - base);
        // bitonic sort of the PLAN_SUB keys, thread t holding positions 2t and 2t + 1:
        // distance 1 inside the thread, 2..64 across the lanes of a wave (shuffles),
        // 128 and more through LDS (10 of the 66 stages need the workgroup barrier)
        uint64_t kk[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = 2 * tid + h;
            kk[h] = ~(uint64_t)0;
            if (i < n) {
                bool bad;
                const int b = plan_bin(d, base + i, K, groups, max_len, total, &bad);
                kk[h] = ((uint64_t)b << 11) | (uint64_t)i;
            }
        }
        for (int k = 2; k <= PLAN_SUB; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                if (j == 1) {
                    const bool up = ((2 * tid) & k) == 0;
                    if ((kk[0] > kk[1]) == up) {
                        const uint64_t t = kk[0];
                        kk[0] = kk[1];
                        kk[1] = t;
                    }
                    continue;
                }
                uint64_t other[2];
                if (j <= 64) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)kk[h], j >> 1, WAVE);
                        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(kk[h] >> 32), j >> 1, WAVE);
                        other[h] = ((uint64_t)hi << 32) | lo;
                    }
                } else {
                    __syncthreads();
                    key[2 * tid] = kk[0];
                    key[2 * tid + 1] = kk[1];
                    __syncthreads();
#pragma unroll
                    for (int h = 0; h < 2; ++h) other[h] = key[(2 * tid + h) ^ j];
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int pp = 2 * tid + h;
                    const bool keep_min = ((pp & j) == 0) == ((pp & k) == 0);
                    kk[h] = keep_min ? (kk[h] < other[h] ? kk[h] : other[h]) : (kk[h] > other[h] ? kk[h] : other[h]);
                }
            }
        }
        __syncthreads();
        key[2 * tid] = kk[0];
        key[2 * tid + 1] = kk[1];
        __syncthreads();
        int last_bin[2] = {-1, -1};
        int last_pos[2] = {0, 0};
        for (int h = 0; h < 2; ++h) {
            const int p = tid + h * 1024;
            if (p >= n) continue;
            const uint64_t kv = key[p];
            const int b = (int)(kv >> 11);
            const uint64_t lo = (uint64_t)b << 11;
            int first = 0, cntp = p;  // first position whose key is >= lo (binary search in [0, p])
            while (first < cntp) {
                const int mid = (first + cntp) >> 1;
                if (key[mid] < lo)
                    first = mid + 1;
                else
                    cntp = mid;
            }
            const int pos = cnt[(int64_t)b * nchunks + c] + (p - first);
            if (dbg_in(pos, S, HMM_DEBUG_PLAN_POS)) perm[pos] = base + (int)(kv & 2047);
            if (p + 1 == n || (int)(key[p + 1] >> 11) != b) {
                last_bin[h] = b;
                last_pos[h] = pos + 1;
            }
        }
        if (base + PLAN_SUB < cend) {
            __syncthreads();  // every cursor of this sub-chunk has been read
            for (int h = 0; h < 2; ++h)
                if (last_bin[h] >= 0) cnt[(int64_t)last_bin[h] * nchunks + c] = last_pos[h];
            __syncthreads();
        }
    }
}

// Chunks of one wave (64 sequences), when the count matrix stays small enough:
// a sequence's rank among the chunk's sequences of its bin comes from ballots,
// one round per distinct bin of the wave (the first unplaced lane's bin, the
// mask of lanes sharing it, the lane's position in that mask).  No LDS and no
// barrier.  Four chunks per block of 256 threads.
__global__ void __launch_bounds__(256) k_plan_scatter_wave(DevPtrs d, int S, int K, int groups, int max_len,
                                                           int64_t total, int nchunks, const int32_t *cnt,
                                                           int32_t *perm) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int c = blockIdx.x * 4 + (int)(threadIdx.x / WAVE);
    if (c >= nchunks) return;  // wave-uniform
    const int s = c * WAVE + lane;
    const bool valid = s < S;
    int b = -1;
    if (valid) {
        bool bad;
        b = plan_bin(d, s, K, groups, max_len, total, &bad);
    }
    const uint64_t below = lane ? (~(uint64_t)0 >> (64 - lane)) : 0;  // lanes under this one
    uint64_t todo = __ballot(valid);
    int rank = 0;
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int lb = __builtin_amdgcn_readlane(b, leader);
        const uint64_t m = __ballot(b == lb);
        if (b == lb) rank = __popcll(m & below);
        todo &= ~m;
    }
    if (valid) {
        const int pos = cnt[(int64_t)b * nchunks + c] + rank;
        if (dbg_in(pos, S, HMM_DEBUG_PLAN_POS)) perm[pos] = s;
    }
}

// cnt_B[k][i][o] for i < N, o < M from the symbol-major emission counts: the
// per-tile partials of model k's tiles summed in tile order (slab), or the
// fixed-point sums; NaN for a model flagged as having received a non-finite
// count.  Tiles of 32 states x 8 symbols through LDS, so both sides are read
// and written in rows; one element per thread, the slab's partials requested 8
// at a time (the sum still takes them in tile order).
__global__ void k_counts_finish_b(AdjLaunch a, int slab, float *cnt_B) {
    __shared__ float tile[8][33];
    const int k = blockIdx.z;
    const int N = a.N, M = a.M, NP = a.NP;
    const int i0 = blockIdx.x * 32, o0 = blockIdx.y * 8;
    const int tx = threadIdx.x, ty = threadIdx.y;
    {
        const int o = o0 + ty, i = i0 + tx;
        float v = 0.0f;
        if (o < M && i < N) {
            if (slab) {
                const int gb = a.gstart[k], ge = a.gstart[k + 1];
                const int nt = (ge - gb + TILE - 1) / TILE;
                const float *src = a.slab + (size_t)slab_slot(gb, k, 0) * M * NP + (size_t)o * NP + i;
                double acc = 0.0;
#pragma unroll 8
                for (int t = 0; t < nt; ++t) acc += (double)src[(size_t)t * M * NP];
                v = (float)acc;
            } else {
                const int F = fixed_exponent(*a.wmax, a.S, a.max_len);
                v = from_fixed(a.B64[((size_t)k * M + o) * NP + quad_t(i)], F);
            }
        }
        tile[ty][tx] = v;
    }
    __syncthreads();
    const bool bad = a.nanflag[k] != 0;
    float *dst = cnt_B + (size_t)k * N * M;
    const int f = ty * 32 + tx;  // 256 threads: state i0 + f / 8, symbol o0 + f % 8
    const int i = i0 + f / 8, o = o0 + f % 8;
    if (i < N && o < M) dst[(size_t)i * M + o] = bad ? __builtin_nanf("") : tile[f % 8][f / 8];
}

// cnt_pi [K][N] and cnt_A [K][N][N] from their fixed-point sums.
__global__ void k_counts_finish_pa(AdjLaunch a, float *cnt_pi, float *cnt_A) {
    const int N = a.N, K = a.K;
    const int F = fixed_exponent(*a.wmax, a.S, a.max_len);
    const int64_t npi = (int64_t)K * N, nA = (int64_t)K * N * N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npi + nA; i += stride) {
        if (i < npi) {
            const int k = (int)(i / N);
            cnt_pi[i] = a.nanflag[k] ? __builtin_nanf("") : from_fixed(a.pi64[i], F);
        } else {
            const int64_t j = i - npi;
            const int k = (int)(j / ((int64_t)N * N));
            cnt_A[j] = a.nanflag[k] ? __builtin_nanf("") : from_fixed(a.A64[j], F);
        }
    }
}

// *wmax = bits of max_s |w_s| over the finite weights (non-negative floats order
// like their bit patterns, so an integer maximum is exact and order-independent).
__global__ void k_weight_max(const float *w, int S, uint32_t *wmax) {
    uint32_t m = 0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
        const float x = fabsf(w[s]);
        if (x <= 3.402823466e38f) m = max(m, __float_as_uint(x));
    }
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0 && m != 0) atomicMax(wmax, m);
}

// Rows of the all-pairs log-likelihoods from the sorted-position staging
// buffer, llpos[k][p] = value of pair (perm[p], k).  One block per 64
// positions, 64 x 64 tiles through LDS: the staging buffer is read along
// positions and out[perm[p]][:] written along models, each row by one wave in
// one pass; the label of each position comes from the same values (smallest
// index of the maximum, NaN skipped, -1 if all NaN).
__global__ void __launch_bounds__(256) k_rows_from_sorted(const float *llpos, const int32_t *perm, int S, int K,
                                                          float *out, int32_t *labels) {
    __shared__ float tile[64][65];  // [position][model]
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int p0 = blockIdx.x * 64;
    const int np = min(64, S - p0);
    int best = -1;
    float bv = 0.0f;
    for (int k0 = 0; k0 < K; k0 += 64) {
        const int nk = min(64, K - k0);
        __syncthreads();
        for (int r = ty; r < nk; r += 4) tile[tx][r] = tx < np ? llpos[(size_t)(k0 + r) * S + p0 + tx] : 0.0f;
        __syncthreads();
        if (labels && ty == 0 && tx < np) {
            for (int r = 0; r < nk; ++r) {
                const float v = tile[tx][r];
                if (v != v) continue;
                if (best < 0 || v > bv) {
                    best = k0 + r;
                    bv = v;
                }
            }
        }
        if (out) {
            for (int r = ty; r < np; r += 4) {
                const int s = perm[p0 + r];
                if (tx < nk) out[(size_t)s * K + k0 + tx] = tile[r][tx];
            }
        }
    }
    if (labels && ty == 0 && tx < np) labels[perm[p0 + tx]] = best;
}

// label[s] = smallest k attaining the maximum of ll[s][:], NaN skipped, -1 if all NaN.
__global__ void k_argmax(const float *ll, int32_t *labels, int S, int K) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const float *row = ll + (size_t)s * K;
    int best = -1;
    float bv = 0.0f;
    for (int k = 0; k < K; ++k) {
        float v = row[k];
        if (v != v) continue;
        if (best < 0 || v > bv) {
            best = k;
            bv = v;
        }
    }
    labels[s] = best;
}

__global__ void k_fill_f32(float *p, size_t n, float v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_copy_i32(const int32_t *src, int32_t *dst, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

// One wave per row.
__global__ void k_softmax_rows(const float *z, float *p, int64_t rows, int cols) {
    int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int lane = threadIdx.x % WAVE;
    if (r >= rows) return;
    const float *zr = z + r * cols;
    float *pr = p + r * cols;
    float m = -INFINITY;
    for (int c = lane; c < cols; c += WAVE) m = fmaxf(m, zr[c]);
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, WAVE));
    float s = 0.0f;
    for (int c = lane; c < cols; c += WAVE) s += expf(zr[c] - m);
    s = wave_sum(s);
    float inv = 1.0f / s;
    for (int c = lane; c < cols; c += WAVE) pr[c] = expf(zr[c] - m) * inv;
}

__global__ void k_logit_grad(const float *n, const float *p, float *g, int64_t rows, int cols) {
    int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int lane = threadIdx.x % WAVE;
    if (r >= rows) return;
    const float *nr = n + r * cols;
    const float *pr = p + r * cols;
    float *gr = g + r * cols;
    float s = 0.0f;
    for (int c = lane; c < cols; c += WAVE) s += nr[c];
    s = wave_sum(s);
    for (int c = lane; c < cols; c += WAVE) gr[c] = nr[c] - pr[c] * s;
}

// Baum-Welch M-step for one parameter array: row r of the expected counts
// divided by its sum; a row whose counts sum to zero keeps its old values.
__global__ void k_reestimate_rows(const float *n, const float *old, float *out, int64_t rows, int cols) {
    int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int lane = threadIdx.x % WAVE;
    if (r >= rows) return;
    const float *nr = n + r * cols;
    const float *orow = old + r * cols;
    float *dst = out + r * cols;
    float s = 0.0f;
    for (int c = lane; c < cols; c += WAVE) s += nr[c];
    s = wave_sum(s);
    if (s > 0.0f) {
        for (int c = lane; c < cols; c += WAVE) dst[c] = nr[c] / s;
    } else {
        for (int c = lane; c < cols; c += WAVE) dst[c] = orow[c];
    }
}

inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }


// Row prefix over a work list: rowpos[p] = rows stored before entry p (the
// lengths of the entries before it, 0 for an invalid sequence), rowpos[S] =
// all rows.  Multi-workgroup form: block sums, their exclusive scan, then each
// workgroup scans its own entries from its block's offset.
constexpr int RP_PER = 8;  // entries per thread
static_assert(ROW_PREFIX_BLOCK == 1024 * RP_PER, "entries per workgroup of the row prefix");

__device__ __forceinline__ int64_t entry_rows(const DevPtrs &d, const RowPrefix &r, int p) {
    const int s = r.perm[p];
    const int32_t T = d.lengths[s];
    return seq_bad(T, d.offsets[s], r.max_len, r.total) ? 0 : (int64_t)T;
}

// Inclusive scan over the 1024 threads of a workgroup; *total gets the sum.
__device__ int64_t block_scan64(int64_t *part, int64_t x, int64_t *total) {
    const int tid = threadIdx.x;
    part[tid] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t y = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    const int64_t res = part[tid];
    *total = part[1023];
    __syncthreads();  // part is free again
    return res;
}

__global__ void __launch_bounds__(1024) k_rows_reduce(DevPtrs d, RowPrefix r) {
    __shared__ int64_t part[1024];
    const int64_t p0 = (int64_t)blockIdx.x * ROW_PREFIX_BLOCK + threadIdx.x;
    int64_t x = 0;
    for (int u = 0; u < RP_PER; ++u) {
        const int64_t p = p0 + (int64_t)u * 1024;
        if (p < r.S) x += entry_rows(d, r, (int)p);
    }
    int64_t tot;
    block_scan64(part, x, &tot);
    if (threadIdx.x == 0) r.rowsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_rows_top(RowPrefix r, int nb) {
    __shared__ int64_t part[1024];
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + (int)threadIdx.x;
        const int64_t x = b < nb ? r.rowsum[b] : 0;
        int64_t tot;
        const int64_t inc = block_scan64(part, x, &tot);
        if (b < nb) r.rowsum[b] = carry + inc - x;
        carry += tot;
    }
}

__global__ void __launch_bounds__(1024) k_rows_apply(DevPtrs d, RowPrefix r, int nb) {
    __shared__ int64_t part[1024];
    const int64_t p0 = (int64_t)blockIdx.x * ROW_PREFIX_BLOCK + (int64_t)threadIdx.x * RP_PER;
    int64_t rows[RP_PER];
    int64_t x = 0;
#pragma unroll
    for (int u = 0; u < RP_PER; ++u) {
        rows[u] = p0 + u < r.S ? entry_rows(d, r, (int)(p0 + u)) : 0;
        x += rows[u];
    }
    int64_t tot;
    int64_t run = block_scan64(part, x, &tot) - x + (nb > 1 ? r.rowsum[blockIdx.x] : 0);
#pragma unroll
    for (int u = 0; u < RP_PER; ++u) {
        if (p0 + u < r.S) r.rowpos[p0 + u] = run;
        run += rows[u];
    }
    if (p0 <= r.S - 1 && r.S - 1 < p0 + RP_PER) r.rowpos[r.S] = run;
    if (blockIdx.x == 0 && (int)threadIdx.x < r.nzero) r.zero[threadIdx.x] = 0;
}

}  // namespace

void plan_chunking(int S, int64_t nbins, int *chunk, int *nchunks) {
    const int64_t nb = nbins > 0 ? nbins : 1;
    const int64_t waves = ((int64_t)S + WAVE - 1) / WAVE;
    if (waves * nb <= PLAN_WAVE_MAX) {  // one wave per chunk
        *chunk = WAVE;
        *nchunks = (int)(waves > 0 ? waves : 1);
        return;
    }
    int64_t nc = ((int64_t)S + PLAN_SUB - 1) / PLAN_SUB;
    const int64_t cap = PLAN_MATRIX_MAX / nb;
    if (nc > cap) nc = cap;
    if (nc < 1) nc = 1;
    int64_t ch = ((int64_t)S + nc - 1) / nc;
    ch = (ch + PLAN_SUB - 1) / PLAN_SUB * PLAN_SUB;
    if (ch < PLAN_SUB) ch = PLAN_SUB;
    *chunk = (int)ch;
    *nchunks = (int)(((int64_t)S + ch - 1) / ch);
    if (*nchunks < 1) *nchunks = 1;
}

void launch_plan(const DevPtrs &d, int K, int S, int groups, int max_len, int64_t total, int nbins,
                 unsigned char *ws, const Layout &L, hipStream_t st, const TransposeJob *tj) {
    int32_t *err = (int32_t *)(ws + L.err);
    int32_t *queue = (int32_t *)(ws + L.queue);
    int32_t *cnt = (int32_t *)(ws + L.hist);
    int32_t *gstart = (int32_t *)(ws + L.gstart);
    int32_t *perm = (int32_t *)(ws + L.perm);
    const int chunk = L.plan_chunk, nchunks = L.plan_nchunks;
    const int64_t n = (int64_t)nbins * nchunks;
    const int64_t m = n > queue_heads(K) ? n : queue_heads(K);
    int nb = blocks_for(m, 256);
    if (nb > 4096) nb = 4096;
    TransposeJob none;
    memset(&none, 0, sizeof(none));
    const TransposeJob &j = tj ? *tj : none;
    hipLaunchKernelGGL(k_plan_init, dim3(nb), dim3(256), 0, st, cnt, n, queue, (int)queue_heads(K), err, j.bmin, K);
    const int count_blocks = blocks_for(S, 256);
    const int tblocks = tj ? transpose_blocks(*tj, K) : 0;
    if (count_blocks + tblocks > 0)
        hipLaunchKernelGGL(k_plan_count, dim3(count_blocks + tblocks), dim3(256), 0, st, d, S, K, groups, max_len,
                           total, chunk, nchunks, cnt, err, count_blocks, j);
    if (n <= PLAN_SCAN_ONE) {
        const size_t dyn = scan_one_lds(n);
        if (dyn > 64 * 1024)
            (void)hipFuncSetAttribute((const void *)k_plan_scan_one, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
        hipLaunchKernelGGL(k_plan_scan_one, dim3(1), dim3(1024), dyn, st, cnt, n, nchunks, max_len + 1, groups, gstart);
    } else {
        const int nscan = (int)((n + PLAN_SCAN - 1) / PLAN_SCAN);
        int32_t *bsum = (int32_t *)(ws + L.scanb);
        hipLaunchKernelGGL(k_plan_scan_reduce, dim3(nscan), dim3(1024), 0, st, cnt, n, bsum);
        hipLaunchKernelGGL(k_plan_scan_top, dim3(1), dim3(1024), 0, st, bsum, nscan);
        hipLaunchKernelGGL(k_plan_scan_apply, dim3(nscan), dim3(1024), 0, st, cnt, n, bsum, nchunks, max_len + 1,
                           groups, gstart);
    }
    if (S > 0 && chunk == WAVE)
        hipLaunchKernelGGL(k_plan_scatter_wave, dim3((nchunks + 3) / 4), dim3(256), 0, st, d, S, K, groups, max_len,
                           total, nchunks, cnt, perm);
    else if (S > 0)
        hipLaunchKernelGGL(k_plan_scatter, dim3(nchunks), dim3(1024), 0, st, d, S, K, groups, max_len, total, chunk,
                           nchunks, cnt, perm);
}

int transpose_blocks(const TransposeJob &j, int K) { return ((j.M + 31) / 32) * ((j.NP + 31) / 32) * K; }

void launch_transpose(const TransposeJob &j, int K, hipStream_t st) {
    if (j.bmin) launch_fill_i32((int32_t *)j.bmin, (size_t)K, 0x7f800000, st);
    hipLaunchKernelGGL(k_transpose, dim3(transpose_blocks(j, K)), dim3(256), 0, st, j);
}

void launch_counts_finish(const AdjLaunch &a, bool slab, float *cnt_pi, float *cnt_A, float *cnt_B, hipStream_t st) {
    const int64_t n = (int64_t)a.K * a.N * (1 + a.N);
    int nb = blocks_for(n, 256);
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_counts_finish_pa, dim3(nb), dim3(256), 0, st, a, cnt_pi, cnt_A);
    dim3 grid((a.N + 31) / 32, (a.M + 7) / 8, a.K);
    hipLaunchKernelGGL(k_counts_finish_b, grid, dim3(32, 8), 0, st, a, slab ? 1 : 0, cnt_B);
}

void launch_weight_max(const float *w, int S, uint32_t *wmax, hipStream_t st) {
    if (w == nullptr) {
        launch_fill_i32((int32_t *)wmax, 1, (int32_t)0x3f800000, st);  // 1.0f: unit weights
        return;
    }
    launch_fill_i32((int32_t *)wmax, 1, 0, st);
    if (S > 0) {
        int nb = blocks_for(S, 256);
        if (nb > 1024) nb = 1024;
        hipLaunchKernelGGL(k_weight_max, dim3(nb), dim3(256), 0, st, w, S, wmax);
    }
}

void launch_rows_from_sorted(const float *llpos, const int32_t *perm, int S, int K, float *out, int32_t *labels,
                             hipStream_t st) {
    if (S > 0)
        hipLaunchKernelGGL(k_rows_from_sorted, dim3(blocks_for(S, 64)), dim3(256), 0, st, llpos, perm, S, K, out, labels);
}

void launch_argmax(const float *ll, int32_t *labels, int S, int K, hipStream_t st) {
    if (S > 0) hipLaunchKernelGGL(k_argmax, dim3(blocks_for(S, 256)), dim3(256), 0, st, ll, labels, S, K);
}

void launch_fill_f32(float *p, size_t n, float v, hipStream_t st) {
    if (n == 0) return;
    int nb = blocks_for((int64_t)n, 256);
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_fill_f32, dim3(nb), dim3(256), 0, st, p, n, v);
}

void launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t st) {
    if (n == 0) return;
    int nb = blocks_for((int64_t)n, 256);
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_fill_i32, dim3(nb), dim3(256), 0, st, p, n, v);
}

void launch_copy_i32(const int32_t *src, int32_t *dst, size_t n, hipStream_t st) {
    if (n == 0) return;
    int nb = blocks_for((int64_t)n, 256);
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_copy_i32, dim3(nb), dim3(256), 0, st, src, dst, n);
}

void launch_softmax_rows(const float *z, float *p, int64_t rows, int cols, hipStream_t st) {
    if (rows > 0) hipLaunchKernelGGL(k_softmax_rows, dim3(blocks_for(rows, 4)), dim3(256), 0, st, z, p, rows, cols);
}

void launch_reestimate_rows(const float *n, const float *old, float *out, int64_t rows, int cols, hipStream_t st) {
    if (rows > 0)
        hipLaunchKernelGGL(k_reestimate_rows, dim3(blocks_for(rows, 4)), dim3(256), 0, st, n, old, out, rows, cols);
}

void launch_logit_grad(const float *n, const float *p, float *g, int64_t rows, int cols, hipStream_t st) {
    if (rows > 0) hipLaunchKernelGGL(k_logit_grad, dim3(blocks_for(rows, 4)), dim3(256), 0, st, n, p, g, rows, cols);
}

hipError_t launch_row_prefix(const DevPtrs &d, const RowPrefix &r, hipStream_t st) {
    if (r.S <= 0 || r.nzero < 0 || r.nzero > 1024) return r.S == 0 ? hipSuccess : hipErrorInvalidValue;
    const int nb = (int)((r.S + (int64_t)ROW_PREFIX_BLOCK - 1) / ROW_PREFIX_BLOCK);
    if (nb > 1) {
        hipLaunchKernelGGL(k_rows_reduce, dim3(nb), dim3(1024), 0, st, d, r);
        hipLaunchKernelGGL(k_rows_top, dim3(1), dim3(1024), 0, st, r, nb);
    }
    hipLaunchKernelGGL(k_rows_apply, dim3(nb), dim3(1024), 0, st, d, r, nb);
    return hipGetLastError();
}

HMM_DEBUG_TAKE(debug_take_planner)

}  // namespace hmm
