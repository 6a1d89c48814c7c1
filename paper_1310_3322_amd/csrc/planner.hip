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

__global__ void k_plan_init(int32_t *cnt, int64_t n, int32_t *queue, int K, int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = i; b < n; b += stride) cnt[b] = 0;
    for (int64_t k = i; k < K; k += stride) queue[k] = 0;
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

__global__ void k_plan_count(DevPtrs d, int S, int K, int groups, int max_len, int64_t total, int chunk,
                             int nchunks, int32_t *cnt, int32_t *err) {
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
    int32_t run = (bsum ? bsum[blockIdx.x] : 0) + block_inclusive_scan(part, local) - local;
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
// sub-chunk) are unique, so the bitonic sort's result is fixed; a sequence's
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
        for (int i = tid; i < PLAN_SUB; i += 1024) {
            uint64_t kv = ~(uint64_t)0;
            if (i < n) {
                bool bad;
                const int b = plan_bin(d, base + i, K, groups, max_len, total, &bad);
                kv = ((uint64_t)b << 11) | (uint64_t)i;
            }
            key[i] = kv;
        }
        __syncthreads();
        for (int k = 2; k <= PLAN_SUB; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int i = (tid / j) * 2 * j + (tid % j);
                const int p = i + j;
                const uint64_t a = key[i], bv = key[p];
                const bool up = (i & k) == 0;
                if ((a > bv) == up) {
                    key[i] = bv;
                    key[p] = a;
                }
                __syncthreads();
            }
        }
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
            perm[pos] = base + (int)(kv & 2047);
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

// Bt[k][o][i] = B[k][i][o] for i < N, 0 for N <= i < NP (32x32 tiles through LDS).
__global__ void k_transpose_b(const float *B, float *bt, int N, int M, int NP) {
    __shared__ float tile[32][33];
    const int k = blockIdx.z;
    const int o0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
    const float *Bk = B + (size_t)k * N * M;
    float *btk = bt + (size_t)k * M * NP;
    for (int r = threadIdx.y; r < 32; r += 8) {
        int i = i0 + r, o = o0 + threadIdx.x;
        tile[r][threadIdx.x] = (i < N && o < M) ? Bk[(size_t)i * M + o] : 0.0f;
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += 8) {
        int o = o0 + r, i = i0 + threadIdx.x;
        if (o < M && i < NP) btk[(size_t)o * NP + i] = tile[threadIdx.x][r];
    }
}

// lnbt[k][o][i] = ln B[k][i][o] for i < N, -inf for N <= i < NP (the emission
// table of the log-domain decoder).
__global__ void k_log_transpose_b(const float *B, float *lnbt, int N, int M, int NP) {
    __shared__ float tile[32][33];
    const int k = blockIdx.z;
    const int o0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
    const float *Bk = B + (size_t)k * N * M;
    float *dst = lnbt + (size_t)k * M * NP;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int i = i0 + r, o = o0 + threadIdx.x;
        tile[r][threadIdx.x] = (i < N && o < M) ? logf(Bk[(size_t)i * M + o]) : -INFINITY;
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int o = o0 + r, i = i0 + threadIdx.x;
        if (o < M && i < NP) dst[(size_t)o * NP + i] = tile[threadIdx.x][r];
    }
}

// cnt_B[k][i][o] for i < N, o < M from the symbol-major emission counts: the
// per-tile partials of model k's tiles summed in tile order (slab), or the
// fixed-point sums; NaN for a model flagged as having received a non-finite
// count.  32 x 32 tiles through LDS, so both sides are read and written in rows.
__global__ void k_counts_finish_b(AdjLaunch a, int slab, float *cnt_B) {
    __shared__ float tile[32][33];
    const int k = blockIdx.z;
    const int N = a.N, M = a.M, NP = a.NP;
    const int i0 = blockIdx.x * 32, o0 = blockIdx.y * 32;
    const int F = fixed_exponent(*a.wmax, a.S, a.max_len);
    const int gb = a.gstart[k], ge = a.gstart[k + 1];
    const int nt = (ge - gb + TILE - 1) / TILE;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int o = o0 + r, i = i0 + threadIdx.x;
        float v = 0.0f;
        if (o < M && i < N) {
            if (slab) {
                const float *src = a.slab + (size_t)slab_slot(gb, k, 0) * M * NP + (size_t)o * NP + i;
                double acc = 0.0;
                for (int t = 0; t < nt; ++t) acc += (double)src[(size_t)t * M * NP];
                v = (float)acc;
            } else {
                v = from_fixed(a.B64[((size_t)k * M + o) * NP + i], F);
            }
        }
        tile[r][threadIdx.x] = v;
    }
    __syncthreads();
    const bool bad = a.nanflag[k] != 0;
    float *dst = cnt_B + (size_t)k * N * M;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int i = i0 + r, o = o0 + threadIdx.x;
        if (i < N && o < M) dst[(size_t)i * M + o] = bad ? __builtin_nanf("") : tile[threadIdx.x][r];
    }
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

}  // namespace

void plan_chunking(int S, int64_t nbins, int *chunk, int *nchunks) {
    int64_t nc = ((int64_t)S + PLAN_SUB - 1) / PLAN_SUB;
    const int64_t cap = PLAN_MATRIX_MAX / (nbins > 0 ? nbins : 1);
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
                 unsigned char *ws, const Layout &L, hipStream_t st) {
    int32_t *err = (int32_t *)(ws + L.err);
    int32_t *queue = (int32_t *)(ws + L.queue);
    int32_t *cnt = (int32_t *)(ws + L.hist);
    int32_t *gstart = (int32_t *)(ws + L.gstart);
    int32_t *perm = (int32_t *)(ws + L.perm);
    const int chunk = L.plan_chunk, nchunks = L.plan_nchunks;
    const int64_t n = (int64_t)nbins * nchunks;
    const int64_t m = n > K ? n : K;
    int nb = blocks_for(m, 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_plan_init, dim3(nb), dim3(256), 0, st, cnt, n, queue, K, err);
    if (S > 0)
        hipLaunchKernelGGL(k_plan_count, dim3(blocks_for(S, 256)), dim3(256), 0, st, d, S, K, groups, max_len, total,
                           chunk, nchunks, cnt, err);
    const int nscan = (int)((n + PLAN_SCAN - 1) / PLAN_SCAN);
    int32_t *bsum = nullptr;
    if (nscan > 1) {
        bsum = (int32_t *)(ws + L.scanb);
        hipLaunchKernelGGL(k_plan_scan_reduce, dim3(nscan), dim3(1024), 0, st, cnt, n, bsum);
        hipLaunchKernelGGL(k_plan_scan_top, dim3(1), dim3(1024), 0, st, bsum, nscan);
    }
    hipLaunchKernelGGL(k_plan_scan_apply, dim3(nscan), dim3(1024), 0, st, cnt, n, bsum, nchunks, max_len + 1, groups,
                       gstart);
    if (S > 0)
        hipLaunchKernelGGL(k_plan_scatter, dim3(nchunks), dim3(1024), 0, st, d, S, K, groups, max_len, total, chunk,
                           nchunks, cnt, perm);
}

void launch_transpose_b(const float *B, float *bt, int K, int N, int M, int NP, hipStream_t st) {
    dim3 grid((M + 31) / 32, (NP + 31) / 32, K);
    hipLaunchKernelGGL(k_transpose_b, grid, dim3(32, 8), 0, st, B, bt, N, M, NP);
}

void launch_log_transpose_b(const float *B, float *lnbt, int K, int N, int M, int NP, hipStream_t st) {
    dim3 grid((M + 31) / 32, (NP + 31) / 32, K);
    hipLaunchKernelGGL(k_log_transpose_b, grid, dim3(32, 8), 0, st, B, lnbt, N, M, NP);
}

void launch_counts_finish(const AdjLaunch &a, bool slab, float *cnt_pi, float *cnt_A, float *cnt_B, hipStream_t st) {
    const int64_t n = (int64_t)a.K * a.N * (1 + a.N);
    int nb = blocks_for(n, 256);
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_counts_finish_pa, dim3(nb), dim3(256), 0, st, a, cnt_pi, cnt_A);
    dim3 grid((a.N + 31) / 32, (a.M + 31) / 32, a.K);
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

}  // namespace hmm
