/*
 * hmm.h — C ABI of libhmm_mi355x.so: a bank of discrete-observation hidden
 * Markov models evaluated over many ragged symbol sequences on one MI355X
 * (gfx950).
 *
 * What is computed.  The paper's activity-recognition stage (Sec. 2.7) keeps
 * one discrete HMM per activity class and provides the Forward, Viterbi and
 * Baum-Welch functions; the HMMs of the different actions are independent and
 * evaluated in parallel (Sec. 3, item 3); an observation is a discretised
 * feature symbol (Sec. 2.5); the configuration knobs are the number of hidden
 * states, the feature-vector size and the number of actions (Sec. 4.1).  The
 * paper prints no formulas; the textbook discrete HMM is used:
 *
 *   pi[k][i]    = P(q_1 = i)                          model k, state i
 *   A[k][i][j]  = P(q_{t+1} = j | q_t = i)            rows sum to 1
 *   B[k][i][o]  = P(o_t = o | q_t = i)                rows sum to 1
 *   alpha_1     = pi o B[:, o_1],   alpha_t = (alpha_{t-1} A) o B[:, o_t]
 *   log P(O | lambda_k) = ln sum_i alpha_T(i)
 *
 * The recursion is renormalised every step (power-of-two rescaling, exact in
 * floating point); the result equals sum_t ln c_t with c_t the per-step sums.
 * Recognition takes the arg-max over models.  The gradient entry point runs the
 * scaled backward (beta) recursion and returns the Baum-Welch E-step expected
 * counts, which are the gradient of sum_s w_s log P(O_s | lambda_{m(s)}) with
 * respect to ln pi, ln A and ln B.
 *
 * Conventions shared by every entry point.
 *  - All array pointers are DEVICE pointers on the current HIP device, owned
 *    by the caller, dense and row-major as declared.  Probabilities are FP32.
 *  - Calls only enqueue work on `stream` and return; results are valid once
 *    the caller synchronises that stream.  No call allocates device memory,
 *    synchronises, or reads device memory back, except hmm_workspace_error
 *    and hmm_debug_flags.
 *    Calls may therefore be captured into a HIP graph.
 *  - Scratch memory is the caller's workspace `ws` of `ws_bytes` bytes, at
 *    least hmm_workspace_size(...) for the same bank, batch and op (Viterbi
 *    decoding and the gradient also take less, see hmm_viterbi and
 *    hmm_forward_backward_grad), 256-byte aligned.  Two calls
 *    in flight at once need two workspaces.
 *  - Host-checkable problems (null pointer, shape out of range, workspace too
 *    small) return a negative status and enqueue nothing.
 *  - Data problems found on the device (a symbol outside [0, M), a negative
 *    length or one above max_len, offset + length outside [0, total_symbols],
 *    a model index outside [0, K)) never cause an out-of-bounds access: the
 *    affected sequence gets NaN log-likelihoods, label -1 and no counts, and
 *    the workspace records the smallest such sequence index
 *    (hmm_workspace_error).
 *  - An impossible observation (a zero per-step sum) gives -inf and no counts.
 *    A sequence of length 0 gives 0 and no counts.
 */
#ifndef HMM_MI355X_H
#define HMM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HMM_OK = 0,
    HMM_ERR_NULL = -1,        /* a required pointer is NULL                        */
    HMM_ERR_SHAPE = -2,       /* K, N, M, S, max_len or total_symbols out of range */
    HMM_ERR_WORKSPACE = -3,   /* workspace NULL, misaligned or too small           */
    HMM_ERR_UNSUPPORTED = -4, /* valid request the library cannot run             */
    HMM_ERR_HIP = -5,         /* a HIP runtime call or kernel launch failed        */
    HMM_ERR_ARG = -6          /* an enumerated argument has an unknown value       */
} hmm_status;

/* A bank of K discrete HMMs with N states and M symbols, FP32 probabilities.
 * 1 <= K <= 65536, 1 <= N <= HMM_MAX_STATES, 1 <= M <= HMM_MAX_SYMBOLS. */
typedef struct {
    int32_t K, N, M;
    const float *pi;   /* [K][N]                                  */
    const float *A;    /* [K][N][N], A[k][i][j] = P(j | i)         */
    const float *B;    /* [K][N][M], B[k][i][o] = P(o | i)         */
} hmm_bank;

/* S ragged int32 symbol sequences.  Sequence s is
 * symbols[offsets[s] .. offsets[s] + lengths[s]).  Sequences may overlap or
 * leave gaps in `symbols`.  max_len (>= every length) and total_symbols (the
 * element count of `symbols`) are host-side promises used to size work; the
 * device checks every sequence against them. */
typedef struct {
    int32_t S;                    /* 0 <= S <= 2^30                                    */
    const int32_t *symbols;       /* [total_symbols], values in [0, M)                 */
    const int64_t *offsets;       /* [S]                                               */
    const int32_t *lengths;       /* [S], 0 <= lengths[s] <= max_len                   */
    const int32_t *model_of_seq;  /* [S] model of each sequence, or NULL = all K models */
    int32_t max_len;              /* 0 <= max_len <= HMM_MAX_LEN                       */
    int64_t total_symbols;        /* >= 0                                              */
} hmm_batch;

#define HMM_MAX_STATES 256
#define HMM_MAX_SYMBOLS 1048576
#define HMM_MAX_LEN 1048576

/* Operation selector for hmm_workspace_size. */
#define HMM_OP_FORWARD 0
#define HMM_OP_CLASSIFY 1
#define HMM_OP_GRAD 2
#define HMM_OP_VITERBI 3

/* Kernel family selector for the forward pass (process-wide; affects later
 * calls).  AUTO and BATCHED choose among the batched families by shape; the
 * last three force one family and make a call return HMM_ERR_UNSUPPORTED when
 * it does not take the shape.  The gradient always uses the batched family
 * that matches its backward kernel. */
#define HMM_KERNEL_AUTO 0     /* batched where supported, else plain                  */
#define HMM_KERNEL_PLAIN 1    /* one wave per (sequence, model) pair                   */
#define HMM_KERNEL_BATCHED 2  /* length-sorted persistent MFMA kernels                 */
#define HMM_KERNEL_TILE16 3   /* one wave per 16-sequence tile (padded N <= 64)        */
#define HMM_KERNEL_TILE32 4   /* one wave per 32-sequence tile (padded N = 32 or 64)   */
#define HMM_KERNEL_COOP 5     /* one workgroup per tile, one wave per state block (N >= 49) */
#define HMM_KERNEL_SCAN 6     /* time-parallel product tree of step matrices, one workgroup
                                 per pair (N <= 16); AUTO takes it for few pairs          */

/* Bytes of workspace the call `op` needs for this bank and batch (host only,
 * reads no device memory; pointers in bank/batch may be NULL here).
 * Returns 0 if the shapes are out of range. */
size_t hmm_workspace_size(const hmm_bank *bank, const hmm_batch *batch, int op);

/* Forward log-likelihoods (Sec. 2.7 "Forward"; Sec. 3 item 3).
 * loglik: [S][K] (sequence-major) when batch->model_of_seq == NULL, else [S];
 * natural log, FP32. */
hmm_status hmm_forward_loglik(const hmm_bank *bank, const hmm_batch *batch, float *loglik,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* Recognition (Sec. 2.7; Fig. 1 output "recognized activity"): every sequence
 * is scored against all K models (model_of_seq is ignored) and
 * labels[s] = smallest k attaining max_k loglik[s][k]; NaN entries are skipped
 * and an all-NaN row gives -1.  loglik_opt: [S][K] or NULL. */
hmm_status hmm_classify(const hmm_bank *bank, const hmm_batch *batch, int32_t *labels,
                        float *loglik_opt, void *ws, size_t ws_bytes, hipStream_t stream);

/* hmm_classify without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture with no workspace prepared,
 * serving loops that must not call the allocator, harnesses that forbid it).
 * The scratch memory is a static device array of HMM_STATIC_SCRATCH_BYTES
 * inside the library: one per GPU, reserved when the library's code is loaded
 * on that GPU and held until the process ends; this call allocates nothing.
 * Arguments, results and errors are those of hmm_classify, plus
 * HMM_ERR_WORKSPACE (nothing enqueued) when hmm_workspace_size(bank, batch,
 * HMM_OP_CLASSIFY) exceeds HMM_STATIC_SCRATCH_BYTES (32 MiB: the 64-model,
 * 65,536-sequence recognition batch with lengths up to 2048 needs 19 MB).
 * Every call on one GPU uses that GPU's one array, which keeps the contents of
 * the last call (each call initialises what it reads): two calls that overlap
 * on one GPU (two streams, two host threads) race and give undefined results. */
#define HMM_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
hmm_status hmm_classify_noalloc(const hmm_bank *bank, const hmm_batch *batch, int32_t *labels,
                                float *loglik_opt, hipStream_t stream);

/* Gradient / Baum-Welch E-step (Sec. 2.7 "BalmWelch") for each sequence with
 * its own model (batch->model_of_seq is required).
 * seq_weight: [S] weight w_s of sequence s (dL/dloglik_s), or NULL = all ones.
 * loglik:     [S] log P(O_s | lambda_{m(s)}).
 * cnt_pi [K][N], cnt_A [K][N][N], cnt_B [K][N][M]: overwritten with
 *   sum_s w_s E[ [q_1 = i] ], sum_s w_s E[ #(i -> j) ], sum_s w_s E[ #(i emits o) ]
 * (the gradient of sum_s w_s loglik_s w.r.t. ln pi, ln A, ln B).
 * phase: 0 = forward and backward in one call;
 *        1 = forward only, writing loglik and keeping the scaled alpha the
 *            backward pass needs in ws (counts untouched, may be NULL);
 *        2 = backward only, from what a phase-1 call with the same bank,
 *            batch, ws and ws_bytes left behind (loglik untouched, may be NULL).
 * Storage of the scaled alpha (the forward variables of Sec. 2.7, rescaled
 * per step) between the passes, chosen by ws_bytes:
 *  - every step: the forward pass stores alphahat_t of every step of every
 *    sequence (one row of NP = padded N floats per step) and the backward pass
 *    reads it back.  Needs a workspace with room for the rows of the batch:
 *    hmm_grad_workspace_size(bank, batch, rows) with rows >= the sum of the
 *    lengths (total_symbols when the sequences do not overlap in `symbols`).
 *    Served for N >= 49; a workspace with fewer rows than the batch needs is
 *    used as below, found on the device without a host synchronisation.
 *  - checkpoints: the forward pass keeps alpha every ceil(sqrt(T)) steps (T
 *    the longest sequence of the length-sorted tile of 16 sequences) and the
 *    backward pass recomputes each segment, so memory grows with sqrt(T) at
 *    the price of a second forward step per step.
 * hmm_workspace_size(..., HMM_OP_GRAD) gives room for every step when the rows
 * take at most 4 GiB, else for checkpoints only.  Both storages give the same
 * counts and log-likelihoods bit for bit.  With every step stored, a phase-0
 * call may overwrite the stored rows during its backward pass (above 128
 * states, or when the emission counts do not fit a workgroup's LDS); phase 2
 * leaves them, so several phase-2 calls may follow one phase-1 call.
 * The counts are deterministic: the same bank, batch and weights give the same
 * counts bit for bit, whatever the tuning choice, the storage or the order in
 * which the device runs the work.  A non-finite weight makes every count of
 * its sequence's model NaN. */
hmm_status hmm_forward_backward_grad(const hmm_bank *bank, const hmm_batch *batch,
                                     const float *seq_weight, float *loglik, float *cnt_pi,
                                     float *cnt_A, float *cnt_B, int32_t phase, void *ws,
                                     size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace with which hmm_forward_backward_grad stores the scaled
 * alpha of `rows` steps (0: checkpoints only; requests above S max_len count
 * as S max_len; ignored below 49 states, where the gradient keeps
 * checkpoints).  Returns 0 if the shapes are out of range or rows < 0.
 * Host only. */
size_t hmm_grad_workspace_size(const hmm_bank *bank, const hmm_batch *batch, int64_t rows);

/* Viterbi decoding (Sec. 2.7 "Viterbi"): the most likely state path of each
 * sequence under its own model (batch->model_of_seq is required), in the log
 * domain:
 *   score[s] = max over state paths Q of ln P(O_s, Q | lambda_{m(s)})   [S], FP32
 *   path[offsets[s] + t] = q_{t+1} of that path, t = 0 .. T_s - 1      [total_symbols], int32
 * (the same layout as the symbols).  Ties are broken towards the smallest
 * state index, both for the last state and for every back-pointer.
 * T = 0 gives score 0; an impossible observation gives score -inf (and the
 * path the tie rule produces); an invalid symbol or model index gives score
 * NaN, path entries -1 and the error word in ws.  Every N up to
 * HMM_MAX_STATES: up to 64 states one wave decodes 64 / N sequences, above a
 * workgroup decodes one sequence.  The traceback reads the FP32 delta row of
 * every step (states padded to 16, 32, 64, 128 or 256; 1 KiB per step at 256
 * states), which the workspace holds for as many steps as it has room for.
 * With room for every row the batch is decoded in one round; otherwise the
 * sequences are decoded longest first in rounds whose rows fit one half of
 * the rows, each round traced back while the next one is decoded in the other
 * half.  Any workspace from hmm_viterbi_workspace_size(bank, batch,
 * min(total_symbols, 2 max_len)) up is accepted (ws_bytes decides the rounds;
 * results do not depend on it).  hmm_workspace_size(..., HMM_OP_VITERBI)
 * gives room for every row when they take at most 4 GiB, else for 1.8 GiB of
 * rows.  The sequences must not overlap in `symbols`: their path entries take
 * the symbols' layout (overlapping sequences may also be left undecoded,
 * reported as invalid). */
hmm_status hmm_viterbi(const hmm_bank *bank, const hmm_batch *batch, float *score, int32_t *path,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace with which hmm_viterbi keeps `rows` delta rows per round
 * (one row per decoded step; rows above total_symbols count as total_symbols).
 * Returns 0 if the shapes are out of range or rows < min(total_symbols,
 * 2 max_len) (one round, or two halves that each hold the longest
 * sequence).  Host only. */
size_t hmm_viterbi_workspace_size(const hmm_bank *bank, const hmm_batch *batch, int64_t rows);

/* Row-wise softmax of FP32 logits: probs[r][c] = exp(z[r][c]) / sum_c' exp(z[r][c']).
 * The parameterisation of the gradient entry point's logits. */
hmm_status hmm_softmax_rows(const float *logits, float *probs, int64_t rows, int32_t cols,
                            hipStream_t stream);

/* Logit gradient from log-probability gradient n and probabilities p
 * (row-wise softmax):  grad[r][c] = n[r][c] - p[r][c] * sum_c' n[r][c']. */
hmm_status hmm_logit_grad(const float *n, const float *probs, float *grad, int64_t rows,
                          int32_t cols, hipStream_t stream);

/* Baum-Welch M-step (Sec. 2.7 "BalmWelch") for one parameter array of `rows`
 * rows of `cols` entries (pi: K rows of N; A: K*N rows of N; B: K*N rows of M):
 *   out[r][c] = n[r][c] / sum_c' n[r][c']   when that sum is > 0,
 *   out[r][c] = old[r][c]                   otherwise (a state or model without counts),
 * where n holds the expected counts of hmm_forward_backward_grad with unit
 * weights.  out may alias old (not n).  One EM iteration is one gradient call
 * followed by this call for pi, A and B. */
hmm_status hmm_reestimate_rows(const float *n, const float *old, float *out, int64_t rows, int32_t cols,
                               hipStream_t stream);

/* The work list the batched kernels of `op` follow (the HMMs of all actions are
 * independent and run side by side, Sec. 3 item 3; the list groups the pairs
 * and sorts them by length so that tiles of consecutive entries advance in
 * step).  order [S]: sequence indices grouped by owning model (one group when
 * op is HMM_OP_CLASSIFY, HMM_OP_FORWARD without model_of_seq or
 * HMM_OP_VITERBI, whose decoders take each sequence's own model), each group
 * sorted by decreasing length, equal lengths in increasing index order (a
 * stable sort, so the list and every tile of it depend on the batch alone).
 * An invalid sequence sorts as length 0 of its group (of group 0 when its model
 * index is out of range) and is recorded in the workspace error word.
 * group_start [groups + 1]: first entry of each group, then S.  Uses the
 * workspace of `op` (hmm_workspace_size); enqueues only, like the calls above. */
hmm_status hmm_plan_order(const hmm_bank *bank, const hmm_batch *batch, int32_t op, int32_t *order,
                          int32_t *group_start, void *ws, size_t ws_bytes, hipStream_t stream);

/* Synchronises `stream`, then reads the workspace error word: *first_bad_seq
 * is the smallest sequence index the last call flagged, or -1 if none. */
hmm_status hmm_workspace_error(const void *ws, hipStream_t stream, int32_t *first_bad_seq);

/* Debug build.  The library built with -DHMM_DEBUG (libhmm_mi355x_debug.so)
 * checks in its kernels the indices it derives for the workspace and the
 * outputs (the bits below); an index outside its buffer is recorded and the
 * access kept inside the buffer or skipped, never made.  hmm_debug_flags
 * synchronises the device, sets *flags to the OR of the bits recorded since
 * the last call and clears them.  A normal build checks nothing and returns
 * HMM_ERR_UNSUPPORTED (*flags = 0).  For tests and diagnosis, not for
 * production: the checks cost time. */
#define HMM_DEBUG_PLAN_POS 1u     /* work-list position outside [0, S)                        */
#define HMM_DEBUG_LL_OUT 2u       /* log-likelihood store outside its output or staging buffer */
#define HMM_DEBUG_CKPT 4u         /* alpha checkpoint outside the sequence's checkpoint slots  */
#define HMM_DEBUG_SLAB 8u         /* per-tile emission partial outside the slab                */
#define HMM_DEBUG_SEGMENT 16u     /* recompute segment longer than the segment buffer          */
#define HMM_DEBUG_VIT_ROWS 32u    /* Viterbi delta rows outside the array (or its half)        */
#define HMM_DEBUG_VIT_ROUND 64u   /* Viterbi round outside the work list                       */
#define HMM_DEBUG_GRAD_ROWS 128u  /* stored alphahat row of the gradient outside its rows      */
hmm_status hmm_debug_flags(uint32_t *flags);

/* Selects the kernel family for later calls (HMM_KERNEL_*).  Any kind other
 * than HMM_KERNEL_AUTO overrides the tuning table below. */
hmm_status hmm_select_kernel(int32_t kind);

/* Tuning table.  The component configuration of Sec. 4.1 leaves the block size
 * of the HMM stage to the user (16 by default); here the knobs are the kernel
 * family (which fixes the tile: 16 or 32 sequences, or a workgroup per tile),
 * the size of the persistent grid and the flags below (where the tile kernels
 * keep the emission table, whether all-pairs tiles are split over the XCDs),
 * picked per call shape by measurement.  While
 * hmm_select_kernel is HMM_KERNEL_AUTO, a call whose shape has an entry takes
 * the entry's choice instead of the built-in heuristics; hmm_workspace_size
 * applies the same entry, so query it after tuning (a choice can need a larger
 * workspace; a call then returns HMM_ERR_WORKSPACE rather than run).  The table
 * lives in host memory, process-wide, at most HMM_TUNE_MAX entries; calls read
 * it on the host only, so they stay capturable into graphs.  Every choice runs
 * kernels held to the same accuracy; the grid cap and the flags change no
 * result, the family may change the rounding of log-likelihoods within that
 * accuracy.  Thread-safe; a call that races with a
 * change of its own entry takes either the old or the new choice. */
#define HMM_TUNE_MAX 256
#define HMM_TUNE_MAX_WG 64
typedef struct {
    int32_t op;         /* HMM_OP_*                                                   */
    int32_t all_pairs;  /* 1: every sequence against every model (classify, or forward
                           without model_of_seq); 0 otherwise                          */
    int32_t K, N, M;    /* bank shape                                                  */
    int32_t s_bucket;   /* bit length of S (0 for S = 0): sizes within a factor 2 share */
    int32_t len_bucket; /* bit length of max_len                                       */
} hmm_tune_key;
typedef struct {
    int32_t kernel;     /* HMM_KERNEL_*; for HMM_OP_GRAD and HMM_OP_VITERBI only AUTO or
                           BATCHED (those ops have one family per shape)             */
    int32_t wg_per_cu;  /* cap on resident workgroups per compute unit of the persistent
                           launches, 0..HMM_TUNE_MAX_WG; 0 = as many as occupancy allows */
    int32_t flags;      /* OR of HMM_TUNE_* below (0 = the built-in rules); they act on the
                           tile forwards (16 and 32 sequences), including the gradient's
                           checkpointing forward                                       */
} hmm_tune_choice;
#define HMM_TUNE_XCD_OFF 1    /* all-pairs tiles not split over the XCDs: each model's tiles in one
                                 queue (default: one queue per XCD when the grid allows)     */
#define HMM_TUNE_BT_GLOBAL 2  /* emission table read from global memory (default: copied into
                                 LDS when it takes at most 48 KB)                             */
#define HMM_TUNE_BT_LDS 4     /* emission table copied into LDS up to 128 KB (fewer workgroups
                                 per CU); not together with HMM_TUNE_BT_GLOBAL                */

/* The key of a call (host only; pointers in bank/batch may be NULL).
 * HMM_ERR_SHAPE / HMM_ERR_ARG for shapes or ops the calls would reject. */
hmm_status hmm_tune_key_of(const hmm_bank *bank, const hmm_batch *batch, int32_t op, hmm_tune_key *key);
/* Installs (replacing) the entry of `key`; choice == NULL removes it.
 * HMM_ERR_ARG for an invalid key or choice, HMM_ERR_UNSUPPORTED when the
 * table is full. */
hmm_status hmm_tune_set(const hmm_tune_key *key, const hmm_tune_choice *choice);
/* *found = 1 and *choice filled when `key` has an entry, else *found = 0. */
hmm_status hmm_tune_get(const hmm_tune_key *key, hmm_tune_choice *choice, int32_t *found);
/* Removes every entry. */
hmm_status hmm_tune_clear(void);
/* The kernel family a call of `op` with this bank and batch would run now,
 * after the selector, the tuning table and the built-in heuristics (host only;
 * pointers may be NULL): HMM_KERNEL_PLAIN, TILE16, TILE32, COOP or SCAN for the
 * forward and classify; TILE16 or COOP for the gradient (the family of its
 * checkpointing forward and backward); BATCHED for Viterbi decoding.
 * HMM_ERR_UNSUPPORTED when the call would return it. */
hmm_status hmm_call_kernel(const hmm_bank *bank, const hmm_batch *batch, int32_t op, int32_t *kernel);

/* Kernel timing for measurement (not needed for computing anything).
 * While enabled, every launch of a main kernel is bracketed by a pair of HIP
 * events recorded on the call's stream (skipped while the stream is being
 * captured into a graph).  hmm_profile_enable(1) clears earlier records;
 * hmm_profile_read synchronises the recorded events and returns, for one
 * kernel family, the summed event-to-event milliseconds and the launch count.
 * Not thread-safe against concurrent calls on other host threads. */
#define HMM_PROF_FWD_BATCHED 0   /* length-sorted MFMA forward            */
#define HMM_PROF_ADJ_BATCHED 1   /* checkpointed MFMA backward            */
#define HMM_PROF_FWD_PLAIN 2     /* plain per-pair forward                */
#define HMM_PROF_VITERBI 3       /* Viterbi decoding and traceback         */
hmm_status hmm_profile_enable(int32_t on);
hmm_status hmm_profile_read(int32_t kernel, double *total_ms, int32_t *launches);

/* Human-readable name of a status code; "HMM_ERR_UNKNOWN" for any other value. */
const char *hmm_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* HMM_MI355X_H */
