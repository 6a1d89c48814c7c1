// Time-parallel forward for the latency regime (gfx950): few, long sequences.
//
// The forward recursion (paper Sec. 2.7 "Forward") is a product of step
// matrices:  alpha_T = alpha_1 M_2 M_3 ... M_T  with  M_t[i][j] = A[i][j] B[j][o_t]
// and alpha_1 = pi o B[:, o_1], so P(O) = alpha_T . 1.  Matrix products are
// associative, so the steps can be multiplied as a balanced tree: the dependent
// chain shrinks from T vector steps to about log2(T) matrix products, for N
// times the work of the recursion.  That trade pays only when the sequences are
// too few to fill the chip with tiles, which is when the batched kernels wait
// on one long sequence.
//
// States are padded to 16.  Pass 1 gives every chunk of 64 steps of every
// (sequence, model) pair its own workgroup: it builds the chunk's step
// matrices in LDS (A_k from registers, the chunk's emission columns staged
// once) and multiplies neighbours level by level in place (pair (i, i + h)
// into slot i); each 16x16 product is four 16x16x4 FP32 MFMAs on one wave,
// rescaled by the power of two of its largest entry, the exponents kept as
// integers.  The chunk product goes to the workspace.  Pass 2, one workgroup
// per pair, reduces the chunk products the same way (64 at a time) and
// advances alpha with each result.  log P = (sum of exponents) ln 2 + ln(sum of
// alpha).
#include <climits>

#include "common.cuh"
#include "kernels.h"

namespace hmm {
namespace {

constexpr int SC_WAVES = 4;
constexpr int SC_ROW = 17;          // padded LDS row (floats) of a 16x16 matrix
constexpr int SC_MAT = 16 * SC_ROW;

__device__ __forceinline__ float wave_max_f(float x) {
    for (int m = 32; m >= 1; m >>= 1) x = fmaxf(x, __shfl_xor(x, m, WAVE));
    return x;
}

struct PairInfo {
    int s, k;
    int32_t T;
    int64_t off;
    bool bad;
};

__device__ __forceinline__ PairInfo pair_info(const DevPtrs &d, const FwdLaunch &f, int64_t p) {
    PairInfo q;
    q.s = f.all_pairs ? (int)(p / f.K) : (int)p;
    q.T = d.lengths[q.s];
    q.off = d.offsets[q.s];
    q.k = f.all_pairs ? (int)(p % f.K) : d.model_of_seq[q.s];
    q.bad = seq_bad(q.T, q.off, f.max_len, f.total) || q.k < 0 || q.k >= f.K;
    return q;
}

// In-place product tree over slots 0 .. n-1 of `mats` (16x16, padded rows) with
// exponents `mexp`: afterwards slot 0 holds the ordered product and its exponent.
__device__ void product_tree(float *mats, int *mexp, int n, int wave, int lane) {
    const int g = lane >> 4, sl = lane & 15;
    for (int h = 1; h < n; h <<= 1) {
        __syncthreads();
        const int npairs = (n - h + 2 * h - 1) / (2 * h);
        for (int pr = wave; pr < npairs; pr += SC_WAVES) {
            const int i = pr * 2 * h, j = i + h;
            const float *X = mats + i * SC_MAT;
            const float *Y = mats + j * SC_MAT;
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const float xa = X[sl * SC_ROW + 4 * kk + g];    // (row sl, k 4kk + g)
                const float yb = Y[(4 * kk + g) * SC_ROW + sl];  // (k 4kk + g, col sl)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, yb, acc, 0, 0, 0);
            }
            float mx = fmaxf(fmaxf(fabsf(acc[0]), fabsf(acc[1])), fmaxf(fabsf(acc[2]), fabsf(acc[3])));
            mx = wave_max_f(mx);
            const int e = frexp_exp(mx);
            float *D = mats + i * SC_MAT;
#pragma unroll
            for (int v = 0; v < 4; ++v) D[(4 * g + v) * SC_ROW + sl] = ldexp_f(acc[v], -e);
            if (lane == 0) mexp[i] = mexp[i] + mexp[j] + e;
        }
    }
    __syncthreads();
}

// The product of the step matrices of steps c0 .. c0 + n - 1 (0-based, n <= 64)
// of pair q into slot 0 of mats (exponent in mexp[0]); *bad_sh is set if one
// of those symbols is outside [0, M).  All threads of the block take part.
__device__ void chunk_product(const DevPtrs &d, const FwdLaunch &f, const PairInfo &q, int c0, int n, float *mats,
                              float (*colb)[16], int *mexp, int *bad_sh) {
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int N = f.N, M = f.M;
    const float *Ak = d.A + (size_t)q.k * N * N;
    const float *Bk = d.B + (size_t)q.k * N * M;
    const int32_t *o = d.symbols + q.off + c0;
    // emission columns of the chunk's symbols
    for (int idx = tid; idx < SCAN_CHUNK * 16; idx += blockDim.x) {
        const int t = idx >> 4, j = idx & 15;
        float v = 0.0f;
        if (t < n) {
            const int ot = o[t];
            if ((unsigned)ot < (unsigned)M) {
                if (j < N) v = Bk[(size_t)j * M + ot];
            } else {
                *bad_sh = 1;
            }
        }
        colb[t][j] = v;
    }
    const int i = tid >> 4, j = tid & 15;  // this thread's entry of every step matrix
    const float a = (i < N && j < N) ? Ak[(size_t)i * N + j] : 0.0f;
    __syncthreads();
    for (int t = 0; t < n; ++t) {
        mats[t * SC_MAT + i * SC_ROW + j] = a * colb[t][j];
        if (tid == 0) mexp[t] = 0;
    }
    product_tree(mats, mexp, n, wave, lane);
}

// Pass 1: block (chunk c, pair p) multiplies the step matrices of steps
// 1 + 64 c .. 1 + 64 c + n - 1 (0-based) and stores the product in
// prod[p][c] (256 floats), its exponent in pexp[p][c] and a bad-symbol flag.
__global__ void __launch_bounds__(SC_WAVES * WAVE) k_scan_chunks(DevPtrs d, FwdLaunch f, ScanWs w) {
    __shared__ float mats[SCAN_CHUNK * SC_MAT];
    __shared__ float colb[SCAN_CHUNK][16];
    __shared__ int mexp[SCAN_CHUNK];
    __shared__ int bad_sh;
    const int tid = threadIdx.x;
    // the error word starts here (pass 2, after this launch, is its only writer)
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *f.err = INT32_MAX;
    const int64_t p = blockIdx.y;
    const int c = blockIdx.x;
    const PairInfo q = pair_info(d, f, p);
    const int c0 = 1 + c * SCAN_CHUNK;
    if (q.bad || c0 >= q.T) return;
    const int n = min(SCAN_CHUNK, q.T - c0);
    if (tid == 0) bad_sh = 0;
    __syncthreads();
    chunk_product(d, f, q, c0, n, mats, colb, mexp, &bad_sh);
    const int i = tid >> 4, j = tid & 15;
    const size_t slot = (size_t)p * w.nch + c;
    w.prod[slot * 256 + tid] = mats[i * SC_ROW + j];
    if (tid == 0) {
        w.pexp[slot] = mexp[0];
        w.pbad[slot] = bad_sh;
    }
}

// alpha_1 = pi o B[:, o_1], rescaled by the power of two of its sum (wave 0;
// returns the exponent).
__device__ int alpha_first(const DevPtrs &d, const FwdLaunch &f, const PairInfo &q, float *alpha, int *bad_sh) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int N = f.N, M = f.M;
    const int o1 = d.symbols[q.off];
    const bool ok = (unsigned)o1 < (unsigned)M;
    if (lane == 0 && !ok) *bad_sh = 1;
    float a = 0.0f;
    if (lane < N && ok) a = d.pi[(size_t)q.k * N + lane] * d.B[((size_t)q.k * N + lane) * M + o1];
    float sum = lane < 16 ? a : 0.0f;
    for (int m = 8; m >= 1; m >>= 1) sum = sum + __shfl_xor(sum, m, WAVE);
    const int e = frexp_exp(sum);
    if (lane < 16) alpha[lane] = ldexp_f(a, -e);
    return e;
}

// alpha <- alpha . P (P: 16x16 in LDS with padded rows), rescaled by the
// power of two of its sum (wave 0; returns the exponent).
__device__ int alpha_advance(float *alpha, const float *P) {
    const int lane = threadIdx.x & (WAVE - 1);
    float u = 0.0f;
    if (lane < 16) {
#pragma clang fp contract(off)
        for (int r = 0; r < 16; ++r) u = u + alpha[r] * P[r * SC_ROW + lane];
    }
    float sum = lane < 16 ? u : 0.0f;
    for (int m = 8; m >= 1; m >>= 1) sum = sum + __shfl_xor(sum, m, WAVE);
    const int e = frexp_exp(sum);
    wave_lds_sync();
    if (lane < 16) alpha[lane] = ldexp_f(u, -e);
    return e;
}

// log P = E ln 2 + ln(sum of alpha) (wave 0, lane 0 writes; NaN and the error
// word for a bad symbol).
__device__ void alpha_finish(const FwdLaunch &f, const PairInfo &q, const float *alpha, int E, int bad, float *out) {
    const int lane = threadIdx.x & (WAVE - 1);
    float a = lane < 16 ? alpha[lane] : 0.0f;
    for (int m = 8; m >= 1; m >>= 1) a = a + __shfl_xor(a, m, WAVE);
    if (lane == 0) {
        float r = (float)((double)E * LN2 + (double)logf(a));
        if (bad) {
            r = NAN;
            atomicMin(f.err, q.s);
        }
        *out = r;
    }
}

__device__ __forceinline__ float *pair_out(const FwdLaunch &f, const PairInfo &q, int64_t p) {
    return f.ll + (f.all_pairs ? (size_t)q.s * f.K + (size_t)(p % f.K) : (size_t)q.s);
}

// Pass 2: block p reduces the chunk products of its pair and advances alpha.
__global__ void __launch_bounds__(SC_WAVES * WAVE) k_scan_combine(DevPtrs d, FwdLaunch f, ScanWs w) {
    __shared__ float mats[SCAN_CHUNK * SC_MAT];
    __shared__ int mexp[SCAN_CHUNK];
    __shared__ float alpha[16];
    __shared__ int bad_sh;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int64_t p = blockIdx.x;
    const PairInfo q = pair_info(d, f, p);
    float *out = pair_out(f, q, p);
    if (q.bad) {
        if (tid == 0) {
            *out = NAN;
            atomicMin(f.err, q.s);
        }
        return;
    }
    if (q.T == 0) {
        if (tid == 0) *out = 0.0f;
        return;
    }
    if (tid == 0) bad_sh = 0;
    int E = 0;
    if (wave == 0) E = alpha_first(d, f, q, alpha, &bad_sh);
    const int nch = (q.T - 1 + SCAN_CHUNK - 1) / SCAN_CHUNK;
    const int i = tid >> 4, j = tid & 15;
    for (int g0 = 0; g0 < nch; g0 += SCAN_CHUNK) {
        const int n = min(SCAN_CHUNK, nch - g0);
        __syncthreads();
        for (int t = 0; t < n; ++t) {
            const size_t slot = (size_t)p * w.nch + g0 + t;
            mats[t * SC_MAT + i * SC_ROW + j] = w.prod[slot * 256 + tid];
            if (tid == 0) {
                mexp[t] = w.pexp[slot];
                if (w.pbad[slot]) bad_sh = 1;
            }
        }
        product_tree(mats, mexp, n, wave, lane);
        if (wave == 0) E += alpha_advance(alpha, mats) + mexp[0];
    }
    __syncthreads();
    if (wave == 0) alpha_finish(f, q, alpha, E, bad_sh, out);
}

// One pair of at most 65 steps (one chunk) in one launch: the chunk product of
// pass 1 and the alpha steps of pass 2 in the same workgroup, with the same
// arithmetic (so the same result) and no workspace traffic.  It also starts the
// error word, which no other block writes.
__global__ void __launch_bounds__(SC_WAVES * WAVE) k_scan_single(DevPtrs d, FwdLaunch f) {
    __shared__ float mats[SCAN_CHUNK * SC_MAT];
    __shared__ float colb[SCAN_CHUNK][16];
    __shared__ int mexp[SCAN_CHUNK];
    __shared__ float alpha[16];
    __shared__ int bad_sh;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    if (tid == 0) *f.err = INT32_MAX;  // the same thread's later atomicMin follows it
    const PairInfo q = pair_info(d, f, 0);
    float *out = pair_out(f, q, 0);
    if (q.bad) {
        if (tid == 0) {
            *out = NAN;
            atomicMin(f.err, q.s);
        }
        return;
    }
    if (q.T == 0) {
        if (tid == 0) *out = 0.0f;
        return;
    }
    if (tid == 0) bad_sh = 0;
    __syncthreads();
    int E = 0;
    if (wave == 0) E = alpha_first(d, f, q, alpha, &bad_sh);
    if (q.T > 1) {
        chunk_product(d, f, q, 1, q.T - 1, mats, colb, mexp, &bad_sh);
        if (wave == 0) E += alpha_advance(alpha, mats) + mexp[0];
    }
    __syncthreads();
    if (wave == 0) alpha_finish(f, q, alpha, E, bad_sh, out);
}

}  // namespace

bool fwd_scan_supported(int N) { return N >= 1 && N <= 16; }

int scan_chunks(int max_len) { return max_len > 1 ? (max_len - 1 + SCAN_CHUNK - 1) / SCAN_CHUNK : 0; }

hipError_t launch_fwd_scan(const DevPtrs &d, const FwdLaunch &f, const ScanWs &w, hipStream_t st) {
    const int64_t pairs = f.all_pairs ? (int64_t)f.S * f.K : (int64_t)f.S;
    if (pairs == 0) {
        launch_fill_i32(f.err, 1, INT32_MAX, st);
        return hipSuccess;
    }
    if (pairs > 65535 && w.nch > 0) return hipErrorInvalidValue;  // grid.y limit of pass 1
    if (pairs > INT_MAX) return hipErrorInvalidValue;
    if (pairs == 1 && w.nch <= 1) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SC_WAVES * WAVE), 0, st, d, f);
        return hipGetLastError();
    }
    if (w.nch == 0) launch_fill_i32(f.err, 1, INT32_MAX, st);
    if (w.nch > 0) {
        hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)w.nch, (unsigned)pairs), dim3(SC_WAVES * WAVE), 0, st, d, f,
                           w);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_combine, dim3((unsigned)pairs), dim3(SC_WAVES * WAVE), 0, st, d, f, w);
    return hipGetLastError();
}

HMM_DEBUG_TAKE(debug_take_fwd_scan)

}  // namespace hmm
