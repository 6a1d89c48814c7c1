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

__global__ void k_plan_init(int32_t *hist, int nbins, int32_t *queue, int K, int32_t *err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int b = i; b < nbins; b += stride) hist[b] = 0;
    for (int k = i; k < K; k += stride) queue[k] = 0;
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

__global__ void k_plan_count(DevPtrs d, int S, int K, int groups, int max_len, int64_t total, int32_t *hist,
                             int32_t *err) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    bool bad;
    int b = plan_bin(d, s, K, groups, max_len, total, &bad);
    atomicAdd(&hist[b], 1);
    if (bad) atomicMin(err, s);
}

// One workgroup of 1024 threads: exclusive scan of the histogram into the
// scatter cursors, plus the start of every group.
__global__ void __launch_bounds__(1024) k_plan_scan(const int32_t *hist, int32_t *cursor, int nbins, int bins_per_group,
                                                    int groups, int32_t *gstart) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int chunk = (nbins + 1023) / 1024;
    const int b0 = min(nbins, tid * chunk), b1 = min(nbins, b0 + chunk);
    int32_t local = 0;
    for (int b = b0; b < b1; ++b) local += hist[b];
    part[tid] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - local;  // exclusive prefix of this chunk
    for (int b = b0; b < b1; ++b) {
        cursor[b] = run;
        if (b % bins_per_group == 0) gstart[b / bins_per_group] = run;
        run += hist[b];
    }
    if (tid == 1023) gstart[groups] = part[1023];
}

__global__ void k_plan_scatter(DevPtrs d, int S, int K, int groups, int max_len, int64_t total, int32_t *cursor,
                               int32_t *perm) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    bool bad;
    int b = plan_bin(d, s, K, groups, max_len, total, &bad);
    int pos = atomicAdd(&cursor[b], 1);
    perm[pos] = s;
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

// cnt_B[k][i][o] = nbt[k][o][i] for i < N: the emission counts accumulated
// symbol-major (one contiguous NP-float row per symbol) back in the caller's
// [K][N][M] layout.
__global__ void k_counts_transpose(const float *nbt, float *cnt_B, int N, int M, int NP) {
    __shared__ float tile[32][33];
    const int k = blockIdx.z;
    const int i0 = blockIdx.x * 32, o0 = blockIdx.y * 32;
    const float *src = nbt + (size_t)k * M * NP;
    float *dst = cnt_B + (size_t)k * N * M;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int o = o0 + r, i = i0 + threadIdx.x;
        tile[r][threadIdx.x] = (o < M && i < N) ? src[(size_t)o * NP + i] : 0.0f;
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int i = i0 + r, o = o0 + threadIdx.x;
        if (i < N && o < M) dst[(size_t)i * M + o] = tile[threadIdx.x][r];
    }
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

void launch_plan(const DevPtrs &d, int K, int S, int groups, int max_len, int64_t total, int nbins,
                 unsigned char *ws, const Layout &L, hipStream_t st) {
    int32_t *err = (int32_t *)(ws + L.err);
    int32_t *queue = (int32_t *)(ws + L.queue);
    int32_t *hist = (int32_t *)(ws + L.hist);
    int32_t *cursor = (int32_t *)(ws + L.cursor);
    int32_t *gstart = (int32_t *)(ws + L.gstart);
    int32_t *perm = (int32_t *)(ws + L.perm);
    int n = nbins > K ? nbins : K;
    int nb = blocks_for(n, 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_plan_init, dim3(nb), dim3(256), 0, st, hist, nbins, queue, K, err);
    if (S > 0)
        hipLaunchKernelGGL(k_plan_count, dim3(blocks_for(S, 256)), dim3(256), 0, st, d, S, K, groups, max_len, total,
                           hist, err);
    hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(1024), 0, st, hist, cursor, nbins, max_len + 1, groups, gstart);
    if (S > 0)
        hipLaunchKernelGGL(k_plan_scatter, dim3(blocks_for(S, 256)), dim3(256), 0, st, d, S, K, groups, max_len,
                           total, cursor, perm);
}

void launch_transpose_b(const float *B, float *bt, int K, int N, int M, int NP, hipStream_t st) {
    dim3 grid((M + 31) / 32, (NP + 31) / 32, K);
    hipLaunchKernelGGL(k_transpose_b, grid, dim3(32, 8), 0, st, B, bt, N, M, NP);
}

void launch_log_transpose_b(const float *B, float *lnbt, int K, int N, int M, int NP, hipStream_t st) {
    dim3 grid((M + 31) / 32, (NP + 31) / 32, K);
    hipLaunchKernelGGL(k_log_transpose_b, grid, dim3(32, 8), 0, st, B, lnbt, N, M, NP);
}

void launch_counts_transpose(const float *nbt, float *cnt_B, int K, int N, int M, int NP, hipStream_t st) {
    dim3 grid((N + 31) / 32, (M + 31) / 32, K);
    hipLaunchKernelGGL(k_counts_transpose, grid, dim3(32, 8), 0, st, nbt, cnt_B, N, M, NP);
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
