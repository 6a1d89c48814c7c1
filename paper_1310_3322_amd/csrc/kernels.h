// Host-side launchers of the HIP kernels (internal to libhmm_mi355x).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.cuh"

namespace hmm {

// Workspace carve-up for one call (byte offsets into ws, 256-aligned).
struct Layout {
    size_t err;      // int32 first bad sequence (INT32_MAX = none)
    size_t queue;    // int32 [K] per-model tile queue heads
    size_t hist;     // int32 [nbins][plan_nchunks] per-chunk bin counts, scanned into placement cursors
    size_t scanb;    // int32 [ceil(nbins * plan_nchunks / 8192)] block sums of that scan
    size_t gstart;   // int32 [groups + 1] start of each group in perm
    size_t perm;     // int32 [S] sequence ids, grouped by model, longest first
    size_t bt;       // float [K][M][NP] transposed, zero-padded emission matrix
    size_t bmin;     // uint32 [K] bits of each model's smallest emission probability (forward)
    size_t ll;       // float [K][S] all-pairs values by sorted position (or [S][K] rows), [S] for the gradient
    size_t ckpt;     // float [S][nck][NP] alpha checkpoints (gradient)
    size_t ckexp;    // int32 [S][nck] exponents of the checkpointed steps
    size_t flag;     // int32 [S] per sorted position: sequence has no finite likelihood
    size_t seg;      // float [slots][seg_stride] segment recompute buffers (gradient)
    size_t pi64;     // uint64 [K][N] fixed-point initial counts (gradient)
    size_t A64;      // uint64 [K][N][N] fixed-point transition counts (gradient)
    size_t B64;      // uint64 [K][M][NP] fixed-point emission counts (gradient, global-count kernels)
    size_t slab;     // float [slab_slots][M][NP] per-tile emission partials (gradient, LDS-partial kernels)
    size_t nanflag;  // int32 [K] models with a non-finite count (gradient)
    size_t wmax;     // uint32 bits of max_s |w_s| (gradient)
    int32_t slab_on;     // the gradient's backward kernel writes per-tile partials into the slab
    size_t frag;     // float4 [K][2][NP^2 / 4] streamed MFMA fragments (cooperative gradient, NP > 128)
    size_t delta;    // float [vit_rows][NP] Viterbi delta rows of one round (bt then holds ln B transposed), then 64 spare floats
    size_t lnat;     // float [K][N][NP] ln A transposed (Viterbi)
    size_t rowpos;   // int64 [S + 1] rows stored before each work-list entry (Viterbi, full-storage gradient)
    size_t rowsum;   // int64 [ceil(S / 8192)] block sums of that prefix
    int64_t grad_rows;   // alphahat rows the gradient may store (0: checkpoints only)
    size_t arow;     // float [grad_rows][NP] alphahat of every step, rows of sorted position p from rowpos[p]
    size_t aexp;     // int32 [grad_rows] exponents of those steps
    size_t mlast;    // float [S] m_T of each sorted position (full-storage gradient)
    // Emission counts from the stored rows (full storage, global-count shapes): the
    // backward pass leaves each live step's weighted gamma in its row, and the rows
    // are grouped by (model, symbol) and summed bucket by bucket instead of with
    // per-step atomics.
    size_t srows;    // uint32 [grad_rows] row indices grouped by bucket
    size_t bucket;   // int32 [K M + 1] first entry of each bucket in srows, then the total
    size_t cursor;   // int32 [K M] rows per bucket, then the scatter cursors
    int64_t vit_rows;    // delta rows one Viterbi round may store
    size_t scan;     // time-parallel forward: chunk products, exponents, flags (ScanWs)
    int32_t scan_nch;    // chunks per pair of the time-parallel forward (0: not used)
    int32_t kind;        // kernel family of the call (HMM_KERNEL_*, after the tuning table)
    int32_t wg_per_cu;   // cap on resident workgroups per CU of persistent launches (0: none)
    int32_t tune_flags;  // HMM_TUNE_* of the call's tuning entry
    size_t total;
    int32_t plan_chunk;    // sequences per chunk of the stable counting sort
    int32_t plan_nchunks;  // chunks of the stable counting sort
    int32_t nck;         // checkpoints per sequence slot
    int32_t seg_slots;   // persistent waves of the gradient kernel
    int64_t seg_stride;  // floats per segment slot
};

// Persistent launches: the occupancy-limited grid, capped at max_grid when
// that is positive (a tuned number of workgroups per CU), reduced when a
// host-side bound on the work items (tiles) is far smaller, so that a small
// batch does not send every resident wave to the same queue counters
// (same-address atomics serialise in L2); then rounded down to a multiple of K
// when it is at least K, so that every model gets the same number of workgroups.
inline int persistent_grid(int occ_grid, int64_t items_bound, int items_per_wg, int K, int max_grid) {
    int grid = (max_grid > 0 && max_grid < occ_grid) ? max_grid : occ_grid;
    occ_grid = grid;
    const int64_t need = (items_bound + items_per_wg - 1) / items_per_wg;
    if (need * 2 < grid) {
        const int64_t floor_k = K < occ_grid ? K : occ_grid;
        grid = (int)(need > floor_k ? need : floor_k);
    }
    if (K > 0 && grid >= K) grid = grid / K * K;
    return grid > 0 ? grid : 1;
}

// XCDs of MI355X; workgroup b of a launch runs on XCD b mod XCDS.
constexpr int XCDS = 8;
// Tile slices of an all-pairs forward: one per XCD when every (model, XCD) pair
// gets at least one workgroup of a grid that divides evenly, else 1.
__host__ __device__ inline int xcd_slices(int all_pairs, int grid, int K) {
    return (all_pairs && grid >= XCDS * K && grid % XCDS == 0) ? XCDS : 1;
}
// Models served by workgroup b of a persistent own-model launch of G
// workgroups: first, first + step, ...  When K and G are multiples of the XCD
// count, the workgroups of XCD x take models x, x + XCDS, ... one after the
// other, sharing each model's tile queue, so that an XCD's L2 holds the tables
// and counts of one model at a time; otherwise workgroup b takes models b mod K
// (or b, b + G, ... when G < K).
__host__ __device__ inline void model_walk(int K, int G, int b, int *first, int *step) {
    if (K % XCDS == 0 && G % XCDS == 0 && G >= K) {
        *first = b % XCDS;
        *step = XCDS;
    } else {
        *first = G >= K ? b % K : b;
        *step = G >= K ? K : G;
    }
}
// Entries of the forward's tile-queue heads: one per model and XCD slice.
__host__ __device__ inline int64_t queue_heads(int K) { return (int64_t)XCDS * K; }

// Upper bound on the tiles of `tile` sequences the planner can form.
inline int64_t tile_bound(int S, int K, bool all_pairs, int tile) {
    const int64_t t = ((int64_t)S + tile - 1) / tile;
    return all_pairs ? t * K : t + K;
}

struct DevPtrs {
    const float *pi, *A, *B;
    const int32_t *symbols;
    const int64_t *offsets;
    const int32_t *lengths;
    const int32_t *model_of_seq;
};

// planner.hip
// Entries of the planner's [bins][chunks] count matrix are capped at this (the
// chunks grow beyond PLAN_SUB sequences when the bins are many).
constexpr int64_t PLAN_MATRIX_MAX = (int64_t)1 << 24;
// With one wave (64 sequences) per chunk the matrix may take up to this many
// entries (128 MiB); beyond it the chunks are sorted in LDS, 2048 at a time.
constexpr int64_t PLAN_WAVE_MAX = (int64_t)1 << 25;
void plan_chunking(int S, int64_t nbins, int *chunk, int *nchunks);
// Emission (or transition) table of every model transposed and padded:
// dst[k][o][i] = B[k][i][o] for i < N (ln of it when lg), 0 (-inf) for N <= i < NP;
// with bmin, bmin[k] = bits of the smallest B[k][i][o].
struct TransposeJob {
    const float *B;
    float *dst;
    int N, M, NP;
    int lg;
    uint32_t *bmin;
};
int transpose_blocks(const TransposeJob &j, int K);
void launch_transpose(const TransposeJob &j, int K, hipStream_t st);
// The plan (and, when tj is given, the transpose in the same launches).
void launch_plan(const DevPtrs &d, int K, int S, int groups, int max_len, int64_t total, int nbins,
                 unsigned char *ws, const Layout &L, hipStream_t st, const TransposeJob *tj = nullptr);
void launch_argmax(const float *ll, int32_t *labels, int S, int K, hipStream_t st);
// out[perm[p]][k] = llpos[k][p] (out may be NULL) and labels[perm[p]] = the arg-max over k
// of the same values (labels may be NULL).
void launch_rows_from_sorted(const float *llpos, const int32_t *perm, int S, int K, float *out, int32_t *labels,
                             hipStream_t st);
void launch_fill_f32(float *p, size_t n, float v, hipStream_t st);
void launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t st);
// Row prefix of a work list (perm[0..S)): rowpos[p] = the lengths of the
// entries before p (0 for an invalid sequence), rowpos[S] = their sum; rowsum
// holds ceil(S / ROW_PREFIX_BLOCK) scratch words; the last kernel also sets
// zero[0..nzero) to 0 (nzero <= 1024).
constexpr int ROW_PREFIX_BLOCK = 8192;
struct RowPrefix {
    const int32_t *perm;
    int S, max_len;
    int64_t total;
    int64_t *rowpos;
    int64_t *rowsum;
    int32_t *zero;
    int nzero;
};
hipError_t launch_row_prefix(const DevPtrs &d, const RowPrefix &r, hipStream_t st);
void launch_copy_i32(const int32_t *src, int32_t *dst, size_t n, hipStream_t st);
void launch_softmax_rows(const float *z, float *p, int64_t rows, int cols, hipStream_t st);
void launch_logit_grad(const float *n, const float *p, float *g, int64_t rows, int cols, hipStream_t st);
void launch_reestimate_rows(const float *n, const float *old, float *out, int64_t rows, int cols, hipStream_t st);

// fwd_plain.hip: one workgroup per (sequence, model) pair
hipError_t launch_fwd_plain(const DevPtrs &d, int K, int N, int M, int S, int all_pairs, int max_len,
                            int64_t total, float *ll, int32_t *err, hipStream_t st);

// fwd_mfma.hip: persistent length-sorted MFMA forward
struct FwdLaunch {
    int K, N, M, NP, S, all_pairs, max_len;
    int64_t total;
    const int32_t *perm, *gstart;
    int32_t *queue, *err;
    const float *bt;
    float *ll;        // [S][K] all pairs (unless llpos), else [S]
    float *llpos;     // [K][S] by sorted position: all-pairs staging, written in tile rows (or NULL)
    const uint32_t *bmin;  // [K] bits of each model's smallest emission probability (or NULL)
    float *ckpt;      // NULL unless checkpointing for the gradient
    int32_t *ckexp;
    int32_t *flag;    // [S] per sorted position: 1 = no finite likelihood (gradient only)
    int nck;
    // Full-storage gradient (arow NULL: checkpoints only): when the rows of all
    // sorted positions fit (rowpos[S] <= grad_rows), every step's alphahat and
    // exponent are stored in place of the checkpoints, and m_T per position.
    float *arow;
    int32_t *aexp;
    float *mlast;
    const int64_t *rowpos;
    int64_t grad_rows;
    int max_grid;     // cap on the persistent grid (0: occupancy limit)
    int tune_flags;   // HMM_TUNE_* of the call
};
// Whether a tile forward copies the emission table (M x NP floats) into LDS.
inline bool bt_in_lds(const FwdLaunch &f) {
    const size_t bytes = (size_t)f.M * f.NP * sizeof(float);
    if (f.tune_flags & HMM_TUNE_BT_GLOBAL) return false;
    return bytes <= ((f.tune_flags & HMM_TUNE_BT_LDS) ? (size_t)128 * 1024 : (size_t)48 * 1024);
}
// The log-likelihood of sequence seq (sorted position pos) under model k.
__device__ __forceinline__ void store_ll(const FwdLaunch &f, int seq, int pos, int k, float r) {
    if (f.llpos) {
        const int64_t i = (int64_t)k * f.S + pos;
        if (dbg_in(i, (int64_t)f.S * f.K, HMM_DEBUG_LL_OUT)) f.llpos[i] = r;
    } else {
        const int64_t i = f.all_pairs ? (int64_t)seq * f.K + k : (int64_t)seq;
        if (dbg_in(i, f.all_pairs ? (int64_t)f.S * f.K : (int64_t)f.S, HMM_DEBUG_LL_OUT)) f.ll[i] = r;
    }
}
bool fwd_mfma_supported(int NP);
hipError_t launch_fwd_mfma(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st);

// fwd_mfma32.hip: persistent length-sorted forward on 32x32x2 MFMA, 32-sequence tiles
bool fwd_mfma32_supported(int NP);
hipError_t launch_fwd_mfma32(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st);

// fwd_scan.hip: time-parallel forward (product tree of step matrices), N <= 16.  Pass 1
// reduces every chunk of SCAN_CHUNK steps of every pair; pass 2 reduces the chunk
// products of each pair.
constexpr int SCAN_CHUNK = 64;
struct ScanWs {
    float *prod;     // [pairs][nch][16][16] chunk products
    int32_t *pexp;   // [pairs][nch] their power-of-two exponents
    int32_t *pbad;   // [pairs][nch] 1 if the chunk holds a symbol outside [0, M)
    int nch;         // chunks per pair (from max_len)
};
bool fwd_scan_supported(int N);
int scan_chunks(int max_len);
hipError_t launch_fwd_scan(const DevPtrs &d, const FwdLaunch &f, const ScanWs &w, hipStream_t st);

// fwd_coop.hip: cooperative-tile forward (one wave per 16-state block)
bool fwd_coop_supported(int NP);
hipError_t launch_fwd_coop(const DevPtrs &d, const FwdLaunch &f, int cu_count, hipStream_t st);

// adj_mfma.hip: checkpointed backward pass producing expected counts
struct AdjLaunch {
    int K, N, M, NP, S, max_len;
    int64_t total;
    const int32_t *perm, *gstart;
    int32_t *queue, *err;
    const float *bt;
    const float *ckpt;
    const int32_t *ckexp;
    const int32_t *flag;
    int nck;
    float *seg;
    int64_t seg_stride;
    int seg_slots;
    const float *weight;
    // Counts, as order-independent 64-bit fixed-point sums (zeroed before the launch):
    unsigned long long *pi64;  // [K][N]
    unsigned long long *A64;   // [K][N][N] n_A = A o C, added tile by tile
    unsigned long long *B64;   // [K][M][NP] symbol-major emission counts (global-count kernels), state i
                               // of a row at quad_t(i)
    float *slab;               // [tiles][M][NP] per-tile emission partials (LDS-partial kernels)
    int32_t *nanflag;          // [K] set when a model received a non-finite count
    const uint32_t *wmax;      // bits of max_s |w_s| (the fixed-point scale)
    const float *frag;  // pre-arranged fragments when the cooperative kernel streams them
    int max_grid;       // cap on the persistent grid (0: occupancy limit)
    // Full-storage gradient (as in FwdLaunch; arow NULL: checkpoints only)
    float *arow;          // the backward pass writes gamma into the rows when srows is set
    uint32_t *srows;      // rows grouped by (model, symbol) (NULL: emission counts by atomics)
    int32_t *bucket, *cursor;
    const int32_t *aexp;
    const float *mlast;
    const int64_t *rowpos;
    int64_t grad_rows;
};
// Whether a gradient call stores every step's alphahat (decided on the device
// from the row prefix, so that overlapping sequences whose rows exceed the
// workspace fall back to checkpoints).
__device__ __forceinline__ bool grad_full(const float *arow, const int64_t *rowpos, int S, int64_t grad_rows) {
    return arow != nullptr && S > 0 && rowpos[S] <= grad_rows;
}
// Quad-transposed position of state i in a row of the global emission counts:
// within each 16-state block, i = 4 g + v goes to 4 v + g.  A lane of the
// backward kernels holds states 4 g + v (v = 0..3) of a sequence, so the four
// lanes of a sequence (g = 0..3) add to four adjacent words in each instruction.
__host__ __device__ inline int quad_t(int i) { return (i & ~15) | ((i & 3) << 2) | ((i >> 2) & 3); }
// Slab slot of tile `tile` of the model whose group starts at gbeg: unique, below
// S / 16 + K + 1 (the group's tiles follow floor(gbeg / 16) + k).
__host__ __device__ inline int64_t slab_slot(int gbeg, int k, int tile) { return (int64_t)(gbeg / 16) + k + tile; }
__host__ __device__ inline int64_t slab_slots(int S, int K) { return (int64_t)S / 16 + K + 1; }
bool adj_mfma_supported(int NP);
// Whether the backward of a shape accumulates emission counts in an LDS partial
// flushed per tile into the slab (true) or in the global fixed-point counts.
bool adj_mfma_slab(int NP, int M, int S, int K);
bool adj_coop_slab(int NP, int M, int S, int K);
// Largest slab of per-tile emission partials a call reserves; beyond it the
// kernels add emission counts to the global fixed-point sums instead.
constexpr int64_t SLAB_MAX_BYTES = (int64_t)1 << 30;
// Final counts: n_pi and n_A from the fixed-point sums, n_B from the slab (tiles of
// each model summed in tile order) or the fixed-point sums, NaN for flagged models.
void launch_counts_finish(const AdjLaunch &a, bool slab, float *cnt_pi, float *cnt_A, float *cnt_B, hipStream_t st);
void launch_weight_max(const float *w, int S, uint32_t *wmax, hipStream_t st);
// adj_coop.hip: cooperative-tile backward (one wave per 16-state block)
bool adj_coop_supported(int NP);
bool adj_coop_streams(int NP);  // fragments streamed from the workspace (launch_coop_frags first)
void launch_coop_frags(const float *A, float *frag, int K, int N, int NP, hipStream_t st);
int adj_coop_slots(int NP, int M, int S, int K, int cu_count);
int64_t adj_coop_seg_stride(int NP, int M, int S, int K, int max_len);
bool adj_coop_pipelined(int NP, int M, int S, int K);  // the two-group pipelined backward serves this shape
hipError_t launch_adj_coop(const DevPtrs &d, const AdjLaunch &a, int cu_count, hipStream_t st);
// Emission counts of the full-storage backward from its gamma rows (a.srows set):
// buckets by (model, symbol), then one wave per bucket sums its rows' fixed-point
// values into a.B64.  Every kernel exits when the call kept checkpoints.
hipError_t launch_counts_from_rows(const DevPtrs &d, const AdjLaunch &a, hipStream_t st);
int adj_mfma_slots(int NP, int M, int S, int K, int cu_count);
int64_t adj_mfma_seg_stride(int NP, int max_len);
hipError_t launch_adj_mfma(const DevPtrs &d, const AdjLaunch &a, int cu_count, hipStream_t st);

// viterbi.hip: max-plus decoding of each sequence with its own model, and its traceback
struct VitLaunch {
    int K, N, M, NP, S, max_len;
    int64_t total;
    const int32_t *perm;     // [S] work list: sequence ids, longest first (all models together)
    const int64_t *rowpos;   // [S + 1] delta rows of the work-list entries before each one
    int64_t *rowsum;         // [ceil(S / 8192)] block sums while rowpos is formed
    int32_t *state;          // [VIT_STATE_WORDS] queue heads and the entries of the current and previous round
    int32_t *err;
    const float *lnbt;  // [K][M][NP] ln B transposed, -inf beyond N
    const float *lnat;  // [K][N][NP] ln A transposed, lnat[k][j][i] = ln A_k[i][j], -inf beyond N
    float *delta;       // [cap_rows][NP] delta rows of the round's sequences, each from its rowpos offset
    float *spill;       // [64] target of the delta stores of empty slots (never read)
    float *score;       // [S]
    int32_t *path;      // [total]
    int64_t cap_rows;   // delta rows the array holds (at least viterbi_min_rows)
    int64_t half_rows;  // rows of each half when rounds alternate halves (0: one round holds every row)
    int max_grid;       // cap on the persistent grid (0: occupancy limit)
};
constexpr int VIT_STATE_WORDS = 9;
bool viterbi_supported(int NP);
int64_t viterbi_min_rows(int64_t max_len, int64_t total);
hipError_t launch_viterbi(const DevPtrs &d, const VitLaunch &v, int cu_count, hipStream_t st);

// Debug build: each translation unit's word of failed bounds checks (taken and cleared).
uint32_t debug_take_planner();
uint32_t debug_take_fwd_plain();
uint32_t debug_take_fwd_mfma();
uint32_t debug_take_fwd_mfma32();
uint32_t debug_take_fwd_coop();
uint32_t debug_take_fwd_scan();
uint32_t debug_take_adj_mfma();
uint32_t debug_take_adj_coop();
uint32_t debug_take_viterbi();
uint32_t debug_take_abi();

}  // namespace hmm
