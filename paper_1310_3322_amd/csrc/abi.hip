// C ABI of libhmm_mi355x: argument checks, workspace carve-up, kernel choice
// and launch order.  Enqueues work only; never allocates, synchronises or
// reads device memory (except hmm_workspace_error, which is documented to).
#include <atomic>
#include <climits>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.cuh"
#include "kernels.h"

using namespace hmm;

namespace {

std::atomic<int> g_kernel_kind{HMM_KERNEL_AUTO};
constexpr int MAX_DEVICES = 64;
std::atomic<int> g_cu_count[MAX_DEVICES];

constexpr int64_t MAX_PLAN_BINS = 1 << 24;

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    if (dev < MAX_DEVICES) {
        int c = g_cu_count[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    if (dev < MAX_DEVICES) g_cu_count[dev].store(n, std::memory_order_relaxed);
    return n;
}

// ---- static scratch area of hmm_classify_noalloc: one array per GPU, in the
// library's code object (reserved by the loader, never by a call).  In host
// code `scratch` only names the array; its device address on the current GPU
// comes from hipGetSymbolAddress, taken once per device on the first call there
// and kept in g_scratch_ptr.  Kernels and fill launches receive that address.
static __device__ __align__(256) unsigned char scratch[HMM_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

hmm_status static_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HMM_ERR_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return HMM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HMM_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HMM_OK;
}

// ---- tuning table (hmm_tune_*): call shape -> kernel family and grid cap
struct TuneEntry {
    hmm_tune_key key;
    hmm_tune_choice choice;
};
std::mutex g_tune_mu;
TuneEntry g_tune[HMM_TUNE_MAX];
int g_tune_n = 0;

int bit_length(int64_t v) {
    int n = 0;
    while (v > 0) {
        ++n;
        v >>= 1;
    }
    return n;
}

bool same_key(const hmm_tune_key &a, const hmm_tune_key &b) {
    return a.op == b.op && a.all_pairs == b.all_pairs && a.K == b.K && a.N == b.N && a.M == b.M &&
           a.s_bucket == b.s_bucket && a.len_bucket == b.len_bucket;
}

hmm_tune_key key_of(const hmm_bank *b, const hmm_batch *q, int op) {
    hmm_tune_key k;
    k.op = op;
    k.all_pairs = (op == HMM_OP_CLASSIFY || (op == HMM_OP_FORWARD && q->model_of_seq == nullptr)) ? 1 : 0;
    k.K = b->K;
    k.N = b->N;
    k.M = b->M;
    k.s_bucket = bit_length(q->S);
    k.len_bucket = bit_length(q->max_len);
    return k;
}

// Kernel family and workgroups per CU of one call: a family forced with
// hmm_select_kernel wins, then the tuning-table entry of the call's shape, then
// the built-in heuristics (AUTO, no cap).
struct CallChoice {
    int kind;
    int wg_per_cu;
    int flags;
};
CallChoice call_choice(const hmm_bank *b, const hmm_batch *q, int op) {
    CallChoice c{g_kernel_kind.load(std::memory_order_relaxed), 0, 0};
    if (c.kind != HMM_KERNEL_AUTO) return c;
    const hmm_tune_key k = key_of(b, q, op);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < g_tune_n; ++i)
        if (same_key(g_tune[i].key, k)) {
            c.kind = g_tune[i].choice.kernel;
            c.wg_per_cu = g_tune[i].choice.wg_per_cu;
            c.flags = g_tune[i].choice.flags;
            break;
        }
    return c;
}

// Grid cap of a call for the persistent launches (0 = none).
int max_grid(int wg_per_cu, int cus) { return wg_per_cu > 0 ? wg_per_cu * cus : 0; }

// ---- optional kernel timing (hmm_profile_*)
struct ProfRecord {
    hipEvent_t start, stop;
    int kind;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_pool;
size_t g_prof_used = 0;

// Records the start event of a main-kernel launch; returns the record index or -1.
int prof_begin(hipStream_t st, int kind) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    if (g_prof_used == g_prof_pool.size()) {
        ProfRecord r;
        if (hipEventCreate(&r.start) != hipSuccess) return -1;
        if (hipEventCreate(&r.stop) != hipSuccess) {
            (void)hipEventDestroy(r.start);
            return -1;
        }
        g_prof_pool.push_back(r);
    }
    const int idx = (int)g_prof_used++;
    g_prof_pool[idx].kind = kind;
    if (hipEventRecord(g_prof_pool[idx].start, st) != hipSuccess) g_prof_pool[idx].kind = -1;
    return idx;
}

void prof_end(hipStream_t st, int idx) {
    if (idx < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (hipEventRecord(g_prof_pool[idx].stop, st) != hipSuccess) g_prof_pool[idx].kind = -1;
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }
inline int pad16(int n) { return ((n + 15) / 16) * 16; }

hmm_status check_shapes(const hmm_bank *b, const hmm_batch *q) {
    if (!b || !q) return HMM_ERR_NULL;
    if (b->K < 1 || b->K > 65536 || b->N < 1 || b->N > HMM_MAX_STATES || b->M < 1 || b->M > HMM_MAX_SYMBOLS)
        return HMM_ERR_SHAPE;
    if (q->S < 0 || q->S > (1 << 30) || q->max_len < 0 || q->max_len > HMM_MAX_LEN || q->total_symbols < 0)
        return HMM_ERR_SHAPE;
    return HMM_OK;
}

hmm_status check_pointers(const hmm_bank *b, const hmm_batch *q) {
    if (!b->pi || !b->A || !b->B) return HMM_ERR_NULL;
    if (q->S > 0 && (!q->offsets || !q->lengths)) return HMM_ERR_NULL;
    if (q->S > 0 && q->total_symbols > 0 && !q->symbols) return HMM_ERR_NULL;
    return HMM_OK;
}

// groups: 1 when every sequence meets every model or, for Viterbi decoding,
// when the work list holds every sequence longest first whatever its model;
// else K
int plan_groups(const hmm_bank *b, const hmm_batch *q, int op) {
    if (op == HMM_OP_CLASSIFY || op == HMM_OP_VITERBI) return 1;
    if (op == HMM_OP_GRAD) return b->K;
    return q->model_of_seq ? b->K : 1;
}

// States padded for the batched kernels: multiples of 16 up to 64 (one wave
// per tile), multiples of 32 above (one wave per 16-state block).
inline int padded_states(int N) { return N <= 64 ? pad16(N) : ((N + 31) / 32) * 32; }

// The gradient's checkpointing forward and its backward must come from the same
// kernel family (the backward recomputes the forward bit for bit): one wave per
// tile up to 48 states, cooperative tiles (one wave per one or two 16-state
// blocks) from 64 to 256 states.
inline bool grad_uses_coop(int NP) { return NP >= 64; }

// States padded for the decoder: lane groups that divide a wave up to 64
// states, a workgroup of 4 threads per state above.
inline int viterbi_states(int N) {
    return N <= 16 ? 16 : N <= 32 ? 32 : N <= 64 ? 64 : N <= 128 ? 128 : N <= 256 ? 256 : 0;
}

bool batched_capable(const hmm_bank *b, const hmm_batch *q, int op) {
    if (op == HMM_OP_VITERBI) return viterbi_states(b->N) > 0 && (int64_t)q->max_len + 1 <= MAX_PLAN_BINS;
    const int NP = padded_states(b->N);
    if (!fwd_mfma_supported(NP) && !fwd_coop_supported(NP)) return false;
    if (op == HMM_OP_GRAD && !(grad_uses_coop(NP) ? adj_coop_supported(NP) : adj_mfma_supported(NP))) return false;
    const int64_t nbins = (int64_t)plan_groups(b, q, op) * ((int64_t)q->max_len + 1);
    return nbins <= MAX_PLAN_BINS;
}

// The time-parallel forward: forced, or chosen for few pairs with long
// sequences, where tiles would leave most of the chip idle while one sequence
// advances step by step.  HMM_ERR_UNSUPPORTED when forced on a shape it does
// not take.
hmm_status scan_choice(const hmm_bank *b, const hmm_batch *q, int op, int kind, bool *scan) {
    *scan = false;
    if (op != HMM_OP_FORWARD && op != HMM_OP_CLASSIFY) return HMM_OK;
    const bool all_pairs = (op == HMM_OP_CLASSIFY) || q->model_of_seq == nullptr;
    const int64_t pairs = all_pairs ? (int64_t)q->S * b->K : (int64_t)q->S;
    if (kind == HMM_KERNEL_SCAN) {
        if (!fwd_scan_supported(b->N) || pairs > 65535) return HMM_ERR_UNSUPPORTED;
        *scan = true;
    } else if (kind == HMM_KERNEL_AUTO) {
        *scan = fwd_scan_supported(b->N) && pairs * 4 <= device_cu_count() && q->max_len >= 32;
    }
    return HMM_OK;
}

// Viterbi delta rows the workspace holds.  Every row (one round) when they
// take at most VIT_ONE_ROUND_BYTES, else VIT_ROUND_BYTES' worth (rounds in
// two halves); never fewer than viterbi_min_rows.
constexpr size_t VIT_ONE_ROUND_BYTES = (size_t)4 << 30;   // 4 GiB
constexpr size_t VIT_ROUND_BYTES = (size_t)1843 << 20;    // 1.8 GiB

int64_t vit_min_rows(const hmm_batch *q) { return viterbi_min_rows(q->max_len, q->total_symbols); }

int64_t vit_max_rows(const hmm_batch *q) {
    const int64_t lo = vit_min_rows(q);
    return q->total_symbols > lo ? q->total_symbols : lo;
}

int64_t vit_default_rows(const hmm_bank *b, const hmm_batch *q) {
    const int NP = viterbi_states(b->N);
    const size_t row = (size_t)(NP > 0 ? NP : 1) * sizeof(float);
    if ((size_t)vit_max_rows(q) * row <= VIT_ONE_ROUND_BYTES) return vit_max_rows(q);
    const int64_t rows = (int64_t)(VIT_ROUND_BYTES / row);
    return rows > vit_min_rows(q) ? rows : vit_min_rows(q);
}

// Alphahat rows of the full-storage gradient (cooperative shapes).  The
// sequences of a batch whose sequences do not overlap in the symbol array need
// at most total_symbols rows; overlapping ones up to S max_len, beyond which
// no request grows.  By default every row of a non-overlapping batch when they
// take at most GRAD_FULL_BYTES, else none (checkpoints only).
constexpr size_t GRAD_FULL_BYTES = (size_t)4 << 30;  // 4 GiB

int64_t grad_max_rows(const hmm_bank *b, const hmm_batch *q) {
    return grad_uses_coop(padded_states(b->N)) ? (int64_t)q->S * q->max_len : 0;
}

int64_t grad_default_rows(const hmm_bank *b, const hmm_batch *q) {
    const int64_t mx = grad_max_rows(b, q);
    const int64_t rows = q->total_symbols < mx ? q->total_symbols : mx;
    const size_t row_bytes = (size_t)padded_states(b->N) * sizeof(float) + sizeof(int32_t);
    return (size_t)rows * row_bytes <= GRAD_FULL_BYTES ? rows : 0;
}

Layout make_layout(const hmm_bank *b, const hmm_batch *q, int op, int64_t vit_rows = -1, int64_t grad_rows = -1) {
    Layout L;
    memset(&L, 0, sizeof(L));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const int K = b->K, M = b->M, S = q->S;
    const int NP = op == HMM_OP_VITERBI ? viterbi_states(b->N) : padded_states(b->N);
    const CallChoice cc = call_choice(b, q, op);
    L.kind = cc.kind;
    L.wg_per_cu = cc.wg_per_cu;
    L.tune_flags = cc.flags;
    L.err = take(64);
    // all pairs: staging buffer of the sorted-position values (or the rows, without a caller buffer)
    if (op == HMM_OP_CLASSIFY || (op == HMM_OP_FORWARD && q->model_of_seq == nullptr))
        L.ll = take((size_t)S * K * sizeof(float));
    if (op == HMM_OP_GRAD) L.ll = take((size_t)S * sizeof(float));
    if (batched_capable(b, q, op)) {
        const int groups = plan_groups(b, q, op);
        const size_t nbins = (size_t)groups * ((size_t)q->max_len + 1);
        L.queue = take((size_t)(queue_heads(K) + K) * sizeof(int32_t));  // forward slices, then the adjoint
        plan_chunking(S, (int64_t)nbins, &L.plan_chunk, &L.plan_nchunks);
        L.hist = take(nbins * (size_t)L.plan_nchunks * sizeof(int32_t));
        L.scanb = take((nbins * (size_t)L.plan_nchunks + 8191) / 8192 * sizeof(int32_t));
        L.gstart = take((size_t)(groups + 1) * sizeof(int32_t));
        L.perm = take((size_t)S * sizeof(int32_t));
        L.bt = take((size_t)K * M * NP * sizeof(float));
        L.bmin = take((size_t)K * sizeof(uint32_t));
        if (op == HMM_OP_VITERBI) {
            L.vit_rows = vit_rows >= 0 ? vit_rows : vit_default_rows(b, q);
            L.delta = take(((size_t)L.vit_rows * NP + 64) * sizeof(float));
            L.lnat = take((size_t)K * b->N * NP * sizeof(float));
            L.rowpos = take(((size_t)S + 1) * sizeof(int64_t));
            L.rowsum = take(((size_t)S + 8191) / 8192 * sizeof(int64_t) + sizeof(int64_t));
        }
        if (op == HMM_OP_GRAD) {
            int nck = 1;
            while ((int64_t)nck * nck < q->max_len) ++nck;
            L.nck = nck;
            L.ckpt = take((size_t)S * nck * NP * sizeof(float));
            L.ckexp = take((size_t)S * nck * sizeof(int32_t));
            L.flag = take((size_t)S * sizeof(int32_t));
            const bool coop = grad_uses_coop(NP);
            const int cus = device_cu_count();
            L.seg_slots = coop ? adj_coop_slots(NP, M, S, K, cus) : adj_mfma_slots(NP, M, S, K, cus);
            L.seg_stride = coop ? adj_coop_seg_stride(NP, M, S, K, q->max_len) : adj_mfma_seg_stride(NP, q->max_len);
            L.seg = take((size_t)L.seg_slots * L.seg_stride * sizeof(float));
            L.slab_on = (coop ? adj_coop_slab(NP, M, S, K) : adj_mfma_slab(NP, M, S, K)) ? 1 : 0;
            L.pi64 = take((size_t)K * b->N * 8);
            L.A64 = take((size_t)K * b->N * b->N * 8);
            if (L.slab_on)
                L.slab = take((size_t)slab_slots(S, K) * M * NP * sizeof(float));
            else
                L.B64 = take((size_t)K * M * NP * 8);
            L.nanflag = take((size_t)K * sizeof(int32_t));
            L.wmax = take(sizeof(uint32_t));
            if (coop && adj_coop_streams(NP)) L.frag = take((size_t)K * 2 * NP * NP * sizeof(float));
            const int64_t mx = grad_max_rows(b, q);
            L.grad_rows = grad_rows < 0 ? grad_default_rows(b, q) : (grad_rows < mx ? grad_rows : mx);
            if (L.grad_rows > 0) {
                L.arow = take((size_t)L.grad_rows * NP * sizeof(float));
                L.aexp = take((size_t)L.grad_rows * sizeof(int32_t));
                L.mlast = take((size_t)S * sizeof(float));
                L.rowpos = take(((size_t)S + 1) * sizeof(int64_t));
                L.rowsum = take(((size_t)S + ROW_PREFIX_BLOCK - 1) / ROW_PREFIX_BLOCK * sizeof(int64_t) + sizeof(int64_t));
                // global-count shapes: emission counts summed from the stored gamma rows by
                // (model, symbol) bucket instead of per-step atomics (32-bit row indices,
                // at most 2^20 buckets)
                const int64_t nbk = (int64_t)K * M;
                if (!L.slab_on && L.grad_rows <= INT32_MAX && nbk <= ((int64_t)1 << 20)) {
                    L.srows = take((size_t)L.grad_rows * sizeof(uint32_t));
                    L.bucket = take(((size_t)nbk + 1) * sizeof(int32_t));
                    L.cursor = take((size_t)nbk * sizeof(int32_t));
                }
            }
        }
    }
    bool scan = false;
    if (scan_choice(b, q, op, L.kind, &scan) == HMM_OK && scan) {
        const bool all_pairs = (op == HMM_OP_CLASSIFY) || q->model_of_seq == nullptr;
        const int64_t pairs = all_pairs ? (int64_t)S * K : (int64_t)S;
        L.scan_nch = scan_chunks(q->max_len);
        const size_t slots = (size_t)pairs * (size_t)L.scan_nch;
        L.scan = take(slots * (256 * sizeof(float) + 2 * sizeof(int32_t)));
    }
    L.total = o;
    return L;
}

hmm_status check_ws(void *ws, size_t ws_bytes, const Layout &L) {
    if (!ws) return HMM_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return HMM_ERR_WORKSPACE;
    if (ws_bytes < L.total) return HMM_ERR_WORKSPACE;
    return HMM_OK;
}

DevPtrs dev_ptrs(const hmm_bank *b, const hmm_batch *q, bool with_models) {
    DevPtrs d;
    d.pi = b->pi;
    d.A = b->A;
    d.B = b->B;
    d.symbols = q->symbols;
    d.offsets = q->offsets;
    d.lengths = q->lengths;
    d.model_of_seq = with_models ? q->model_of_seq : nullptr;
    return d;
}

// Chooses the family for a call; HMM_ERR_UNSUPPORTED when the batched family
// is forced for a shape it does not take.
hmm_status choose(const hmm_bank *b, const hmm_batch *q, int op, int kind, bool *batched) {
    const bool cap = batched_capable(b, q, op);
    if (op == HMM_OP_GRAD) {
        if (!cap) return HMM_ERR_UNSUPPORTED;
        *batched = true;
        return HMM_OK;
    }
    if (kind == HMM_KERNEL_PLAIN) {
        *batched = false;
        return HMM_OK;
    }
    if (kind >= HMM_KERNEL_BATCHED && !cap) return HMM_ERR_UNSUPPORTED;
    *batched = cap;
    return HMM_OK;
}

// The concrete forward family of a call (HMM_KERNEL_PLAIN, TILE16, TILE32,
// COOP or SCAN) under the call's kind; HMM_ERR_UNSUPPORTED when a forced
// family does not take the shape.  Host only, decided before anything is
// enqueued.
hmm_status forward_family(const hmm_bank *b, const hmm_batch *q, int op, int kind, int *fam) {
    bool batched = false;
    hmm_status rc = choose(b, q, op, kind, &batched);
    if (rc != HMM_OK) return rc;
    if (!batched) {
        *fam = HMM_KERNEL_PLAIN;
        return HMM_OK;
    }
    bool scan = false;
    if ((rc = scan_choice(b, q, op, kind, &scan)) != HMM_OK) return rc;
    if (scan) {
        *fam = HMM_KERNEL_SCAN;
        return HMM_OK;
    }
    const bool all_pairs = (op == HMM_OP_CLASSIFY) || q->model_of_seq == nullptr;
    const int K = b->K, S = q->S, NP = padded_states(b->N);
    const int cus = device_cu_count();
    // One wave per tile while the tiles fill the chip; one wave per 16-state
    // block (cooperative tile) when the state count needs it or tiles are few.
    const int64_t tiles = ((int64_t)S + TILE - 1) / TILE + (all_pairs ? 0 : K);
    const int64_t items = all_pairs ? tiles * K : tiles;
    bool coop = !fwd_mfma_supported(NP) || (fwd_coop_supported(NP) && items < (int64_t)8 * cus);
    // 32-sequence tiles halve the per-state vector work when there are enough of them
    const int64_t items32 = all_pairs ? (((int64_t)S + 31) / 32) * K : ((int64_t)S + 31) / 32 + K;
    bool wide = !coop && fwd_mfma32_supported(NP) && items32 >= (int64_t)8 * cus;
    if (kind == HMM_KERNEL_TILE16) {
        if (!fwd_mfma_supported(NP)) return HMM_ERR_UNSUPPORTED;
        coop = wide = false;
    } else if (kind == HMM_KERNEL_TILE32) {
        if (!fwd_mfma32_supported(NP)) return HMM_ERR_UNSUPPORTED;
        coop = false;
        wide = true;
    } else if (kind == HMM_KERNEL_COOP) {
        if (!fwd_coop_supported(NP)) return HMM_ERR_UNSUPPORTED;
        coop = true;
        wide = false;
    }
    *fam = coop ? HMM_KERNEL_COOP : (wide ? HMM_KERNEL_TILE32 : HMM_KERNEL_TILE16);
    return HMM_OK;
}

// The forward of a call, then, for recognition, the labels.  out: [S][K] all
// pairs or [S]; may be NULL for recognition (labels only).  The length-sorted
// families write all-pairs values by sorted position into the workspace's
// staging buffer (rows of each tile contiguous) and one pass writes the
// caller's rows and the labels from it; the plain and time-parallel kernels
// write the rows directly (into the staging buffer when out is NULL).
hmm_status run_forward(const hmm_bank *b, const hmm_batch *q, int op, float *out, int32_t *labels, unsigned char *ws,
                       const Layout &L, hipStream_t st) {
    const bool all_pairs = (op == HMM_OP_CLASSIFY) || q->model_of_seq == nullptr;
    int fam = HMM_KERNEL_PLAIN;
    hmm_status rc = forward_family(b, q, op, L.kind, &fam);
    if (rc != HMM_OK) return rc;
    const bool batched = fam != HMM_KERNEL_PLAIN;
    DevPtrs d = dev_ptrs(b, q, !all_pairs);
    int32_t *err = (int32_t *)(ws + L.err);
    const int K = b->K, N = b->N, M = b->M, S = q->S;
    float *staging = all_pairs ? (float *)(ws + L.ll) : nullptr;
    float *direct = out ? out : staging;  // target of the kernels that write rows themselves
    auto finish_direct = [&](hipError_t e) {
        if (e != hipSuccess) return HMM_ERR_HIP;
        if (labels) launch_argmax(direct, labels, S, K, st);
        return hipGetLastError() == hipSuccess ? HMM_OK : HMM_ERR_HIP;
    };
    if (!batched) {
        launch_fill_i32(err, 1, INT32_MAX, st);
        const int pr = prof_begin(st, HMM_PROF_FWD_PLAIN);
        const hipError_t e = launch_fwd_plain(d, K, N, M, S, all_pairs ? 1 : 0, q->max_len, q->total_symbols, direct,
                                              err, st);
        prof_end(st, pr);
        return finish_direct(e);
    }
    const int NP = padded_states(N);
    const int cus = device_cu_count();
    {
        if (fam == HMM_KERNEL_SCAN) {  // (the time-parallel kernels start the error word themselves)
            FwdLaunch f;
            memset(&f, 0, sizeof(f));
            f.K = K;
            f.N = N;
            f.M = M;
            f.NP = 16;
            f.S = S;
            f.all_pairs = all_pairs ? 1 : 0;
            f.max_len = q->max_len;
            f.total = q->total_symbols;
            f.err = err;
            f.ll = direct;
            const int64_t pairs = all_pairs ? (int64_t)S * K : (int64_t)S;
            ScanWs sw;
            sw.nch = L.scan_nch;
            sw.prod = (float *)(ws + L.scan);
            sw.pexp = (int32_t *)(sw.prod + (size_t)pairs * sw.nch * 256);
            sw.pbad = sw.pexp + (size_t)pairs * sw.nch;
            const int pr = prof_begin(st, HMM_PROF_FWD_BATCHED);
            const hipError_t e = launch_fwd_scan(d, f, sw, st);
            prof_end(st, pr);
            return finish_direct(e);
        }
    }
    const int groups = all_pairs ? 1 : K;
    const int nbins = groups * (q->max_len + 1);
    const TransposeJob tj{b->B, (float *)(ws + L.bt), N, M, NP, 0, (uint32_t *)(ws + L.bmin)};
    launch_plan(d, K, S, groups, q->max_len, q->total_symbols, nbins, ws, L, st, &tj);
    if (hipGetLastError() != hipSuccess) return HMM_ERR_HIP;
    FwdLaunch f;
    memset(&f, 0, sizeof(f));
    f.K = K;
    f.N = N;
    f.M = M;
    f.NP = NP;
    f.S = S;
    f.all_pairs = all_pairs ? 1 : 0;
    f.max_len = q->max_len;
    f.total = q->total_symbols;
    f.perm = (const int32_t *)(ws + L.perm);
    f.gstart = (const int32_t *)(ws + L.gstart);
    f.queue = (int32_t *)(ws + L.queue);
    f.err = err;
    f.bt = (const float *)(ws + L.bt);
    f.ll = out;
    f.llpos = staging;
    f.bmin = (const uint32_t *)(ws + L.bmin);
    f.max_grid = max_grid(L.wg_per_cu, cus);
    f.tune_flags = L.tune_flags;
    if (S == 0) return HMM_OK;
    const int pr = prof_begin(st, HMM_PROF_FWD_BATCHED);
    const hipError_t e = fam == HMM_KERNEL_COOP    ? launch_fwd_coop(d, f, cus, st)
                         : fam == HMM_KERNEL_TILE32 ? launch_fwd_mfma32(d, f, cus, st)
                                                    : launch_fwd_mfma(d, f, cus, st);
    prof_end(st, pr);
    if (e != hipSuccess) return HMM_ERR_HIP;
    if (all_pairs) launch_rows_from_sorted(staging, f.perm, S, K, out, labels, st);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_ERR_HIP;
}

}  // namespace

namespace hmm {
HMM_DEBUG_TAKE(debug_take_abi)
}  // namespace hmm

extern "C" {

size_t hmm_workspace_size(const hmm_bank *bank, const hmm_batch *batch, int op) {
    if (op < HMM_OP_FORWARD || op > HMM_OP_VITERBI) return 0;
    if (check_shapes(bank, batch) != HMM_OK) return 0;
    return make_layout(bank, batch, op).total;
}

hmm_status hmm_forward_loglik(const hmm_bank *bank, const hmm_batch *batch, float *loglik, void *ws,
                              size_t ws_bytes, hipStream_t stream) {
    hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    if ((rc = check_pointers(bank, batch)) != HMM_OK) return rc;
    if (batch->S > 0 && !loglik) return HMM_ERR_NULL;
    const Layout L = make_layout(bank, batch, HMM_OP_FORWARD);
    if ((rc = check_ws(ws, ws_bytes, L)) != HMM_OK) return rc;
    return run_forward(bank, batch, HMM_OP_FORWARD, loglik, nullptr, (unsigned char *)ws, L, stream);
}

hmm_status hmm_classify_noalloc(const hmm_bank *bank, const hmm_batch *batch, int32_t *labels,
                                float *loglik_opt, hipStream_t stream) {
    hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    if (make_layout(bank, batch, HMM_OP_CLASSIFY).total > HMM_STATIC_SCRATCH_BYTES) return HMM_ERR_WORKSPACE;
    void *ws = nullptr;
    if ((rc = static_scratch(&ws)) != HMM_OK) return rc;
    return hmm_classify(bank, batch, labels, loglik_opt, ws, HMM_STATIC_SCRATCH_BYTES, stream);
}

hmm_status hmm_classify(const hmm_bank *bank, const hmm_batch *batch, int32_t *labels, float *loglik_opt,
                        void *ws, size_t ws_bytes, hipStream_t stream) {
    hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    if ((rc = check_pointers(bank, batch)) != HMM_OK) return rc;
    if (batch->S > 0 && !labels) return HMM_ERR_NULL;
    const Layout L = make_layout(bank, batch, HMM_OP_CLASSIFY);
    if ((rc = check_ws(ws, ws_bytes, L)) != HMM_OK) return rc;
    return run_forward(bank, batch, HMM_OP_CLASSIFY, loglik_opt, labels, (unsigned char *)ws, L, stream);
}

// Alphahat rows of the largest gradient layout that fits ws_bytes (0 when only
// the checkpoint layout fits, -1 when not even that does).
int64_t grad_rows_for(const hmm_bank *b, const hmm_batch *q, size_t ws_bytes) {
    int64_t lo = 0, hi = grad_max_rows(b, q);
    if (make_layout(b, q, HMM_OP_GRAD, -1, lo).total > ws_bytes) return -1;
    if (make_layout(b, q, HMM_OP_GRAD, -1, hi).total <= ws_bytes) return hi;
    while (hi - lo > 1) {  // the layout grows with the rows: fits at lo, not at hi
        const int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(b, q, HMM_OP_GRAD, -1, mid).total <= ws_bytes)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

size_t hmm_grad_workspace_size(const hmm_bank *bank, const hmm_batch *batch, int64_t rows) {
    if (check_shapes(bank, batch) != HMM_OK) return 0;
    if (rows < 0) return 0;
    return make_layout(bank, batch, HMM_OP_GRAD, -1, rows).total;
}

hmm_status hmm_forward_backward_grad(const hmm_bank *bank, const hmm_batch *batch, const float *seq_weight,
                                     float *loglik, float *cnt_pi, float *cnt_A, float *cnt_B, int32_t phase,
                                     void *ws, size_t ws_bytes, hipStream_t stream) {
    hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    if (phase < 0 || phase > 2) return HMM_ERR_ARG;
    if ((rc = check_pointers(bank, batch)) != HMM_OK) return rc;
    if (batch->S > 0 && !batch->model_of_seq) return HMM_ERR_NULL;
    if (phase != 1 && (!cnt_pi || !cnt_A || !cnt_B)) return HMM_ERR_NULL;
    // the stored alphahat rows: as many as the workspace holds
    const int64_t rows = grad_rows_for(bank, batch, ws ? ws_bytes : 0);
    const Layout L = make_layout(bank, batch, HMM_OP_GRAD, -1, rows < 0 ? 0 : rows);
    if ((rc = check_ws(ws, ws_bytes, L)) != HMM_OK) return rc;
    bool batched = false;
    if ((rc = choose(bank, batch, HMM_OP_GRAD, L.kind, &batched)) != HMM_OK) return rc;
    unsigned char *w = (unsigned char *)ws;
    const int K = bank->K, N = bank->N, M = bank->M, S = batch->S, NP = padded_states(N);
    DevPtrs d = dev_ptrs(bank, batch, true);
    int32_t *err = (int32_t *)(w + L.err);
    float *ll = loglik ? loglik : (float *)(w + L.ll);
    const int cus = device_cu_count();
    if (phase != 2) {
        const int nbins = K * (batch->max_len + 1);
        const TransposeJob tj{bank->B, (float *)(w + L.bt), N, M, NP, 0, nullptr};
        launch_plan(d, K, S, K, batch->max_len, batch->total_symbols, nbins, w, L, stream, &tj);
        if (hipGetLastError() != hipSuccess) return HMM_ERR_HIP;
        if (L.grad_rows > 0) {  // first stored row of each sorted position
            const RowPrefix rp{(const int32_t *)(w + L.perm), S, batch->max_len, batch->total_symbols,
                               (int64_t *)(w + L.rowpos), (int64_t *)(w + L.rowsum), nullptr, 0};
            if (launch_row_prefix(d, rp, stream) != hipSuccess) return HMM_ERR_HIP;
        }
        FwdLaunch f;
        memset(&f, 0, sizeof(f));
        f.K = K;
        f.N = N;
        f.M = M;
        f.NP = NP;
        f.S = S;
        f.all_pairs = 0;
        f.max_len = batch->max_len;
        f.total = batch->total_symbols;
        f.perm = (const int32_t *)(w + L.perm);
        f.gstart = (const int32_t *)(w + L.gstart);
        f.queue = (int32_t *)(w + L.queue);
        f.err = err;
        f.bt = (const float *)(w + L.bt);
        f.ll = ll;
        f.ckpt = (float *)(w + L.ckpt);
        f.ckexp = (int32_t *)(w + L.ckexp);
        f.flag = (int32_t *)(w + L.flag);
        f.nck = L.nck;
        if (L.grad_rows > 0) {
            f.arow = (float *)(w + L.arow);
            f.aexp = (int32_t *)(w + L.aexp);
            f.mlast = (float *)(w + L.mlast);
            f.rowpos = (const int64_t *)(w + L.rowpos);
            f.grad_rows = L.grad_rows;
        }
        f.max_grid = max_grid(L.wg_per_cu, cus);
        f.tune_flags = L.tune_flags;
        if (S > 0) {
            const int pr = prof_begin(stream, HMM_PROF_FWD_BATCHED);
            const hipError_t e = grad_uses_coop(NP) ? launch_fwd_coop(d, f, cus, stream) : launch_fwd_mfma(d, f, cus, stream);
            prof_end(stream, pr);
            if (e != hipSuccess) return HMM_ERR_HIP;
        }
    }
    if (phase == 1) return HMM_OK;
    const bool coop = grad_uses_coop(NP);
    const bool slab = L.slab_on != 0;
    // the fixed-point count sums start at zero (fill kernels: no memset nodes in a captured graph)
    launch_fill_i32((int32_t *)(w + L.pi64), (size_t)2 * K * N, 0, stream);
    launch_fill_i32((int32_t *)(w + L.A64), (size_t)2 * K * N * N, 0, stream);
    if (!slab) launch_fill_i32((int32_t *)(w + L.B64), (size_t)2 * K * M * NP, 0, stream);
    launch_fill_i32((int32_t *)(w + L.nanflag), (size_t)K, 0, stream);
    launch_weight_max(seq_weight, S, (uint32_t *)(w + L.wmax), stream);
    int32_t *queue2 = (int32_t *)(w + L.queue) + queue_heads(K);
    launch_fill_i32(queue2, (size_t)K, 0, stream);
    if (hipGetLastError() != hipSuccess) return HMM_ERR_HIP;
    AdjLaunch a;
    memset(&a, 0, sizeof(a));
    a.K = K;
    a.N = N;
    a.M = M;
    a.NP = NP;
    a.S = S;
    a.max_len = batch->max_len;
    a.total = batch->total_symbols;
    a.perm = (const int32_t *)(w + L.perm);
    a.gstart = (const int32_t *)(w + L.gstart);
    a.queue = queue2;
    a.err = err;
    a.bt = (const float *)(w + L.bt);
    a.ckpt = (const float *)(w + L.ckpt);
    a.ckexp = (const int32_t *)(w + L.ckexp);
    a.flag = (const int32_t *)(w + L.flag);
    a.nck = L.nck;
    a.seg = (float *)(w + L.seg);
    a.seg_stride = L.seg_stride;
    a.seg_slots = L.seg_slots;
    a.weight = seq_weight;
    a.pi64 = (unsigned long long *)(w + L.pi64);
    a.A64 = (unsigned long long *)(w + L.A64);
    a.B64 = slab ? nullptr : (unsigned long long *)(w + L.B64);
    a.slab = slab ? (float *)(w + L.slab) : nullptr;
    a.nanflag = (int32_t *)(w + L.nanflag);
    a.wmax = (const uint32_t *)(w + L.wmax);
    a.max_grid = max_grid(L.wg_per_cu, cus);
    if (L.grad_rows > 0) {
        a.arow = (float *)(w + L.arow);
        // the walk overwrites the rows with gamma, so only a call that ran its own
        // forward does (a phase-2 call leaves them for the next phase 2)
        if (L.srows && phase == 0) {
            a.srows = (uint32_t *)(w + L.srows);
            a.bucket = (int32_t *)(w + L.bucket);
            a.cursor = (int32_t *)(w + L.cursor);
        }
        a.aexp = (const int32_t *)(w + L.aexp);
        a.mlast = (const float *)(w + L.mlast);
        a.rowpos = (const int64_t *)(w + L.rowpos);
        a.grad_rows = L.grad_rows;
    }
    if (S > 0) {
        if (coop && adj_coop_streams(NP)) {
            float *frag = (float *)(w + L.frag);
            launch_coop_frags(bank->A, frag, K, N, NP, stream);
            a.frag = frag;
        }
        const int pr = prof_begin(stream, HMM_PROF_ADJ_BATCHED);
        hipError_t e = coop ? launch_adj_coop(d, a, cus, stream) : launch_adj_mfma(d, a, cus, stream);
        if (e == hipSuccess && coop) e = launch_counts_from_rows(d, a, stream);
        prof_end(stream, pr);
        if (e != hipSuccess) return HMM_ERR_HIP;
    }
    launch_counts_finish(a, slab, cnt_pi, cnt_A, cnt_B, stream);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_ERR_HIP;
}

// Delta rows of the largest Viterbi layout that fits ws_bytes (every row at
// most), or -1 when not even the smallest fits.
int64_t vit_rows_for(const hmm_bank *b, const hmm_batch *q, size_t ws_bytes) {
    int64_t lo = vit_min_rows(q), hi = vit_max_rows(q);
    if (make_layout(b, q, HMM_OP_VITERBI, lo).total > ws_bytes) return -1;
    if (make_layout(b, q, HMM_OP_VITERBI, hi).total <= ws_bytes) return hi;
    while (hi - lo > 1) {  // the layout grows with the rows: fits at lo, not at hi
        const int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(b, q, HMM_OP_VITERBI, mid).total <= ws_bytes)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

size_t hmm_viterbi_workspace_size(const hmm_bank *bank, const hmm_batch *batch, int64_t rows) {
    if (check_shapes(bank, batch) != HMM_OK) return 0;
    if (rows < vit_min_rows(batch)) return 0;
    if (rows > vit_max_rows(batch)) rows = vit_max_rows(batch);
    return make_layout(bank, batch, HMM_OP_VITERBI, rows).total;
}

hmm_status hmm_viterbi(const hmm_bank *bank, const hmm_batch *batch, float *score, int32_t *path, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
    hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    if ((rc = check_pointers(bank, batch)) != HMM_OK) return rc;
    if (batch->S > 0 && (!batch->model_of_seq || !score)) return HMM_ERR_NULL;
    if (batch->total_symbols > 0 && !path) return HMM_ERR_NULL;
    if (!batched_capable(bank, batch, HMM_OP_VITERBI)) return HMM_ERR_UNSUPPORTED;
    // the delta rows of a round: as many as the workspace holds
    const int64_t rows = vit_rows_for(bank, batch, ws ? ws_bytes : 0);
    const Layout L = make_layout(bank, batch, HMM_OP_VITERBI, rows < 0 ? vit_min_rows(batch) : rows);
    if ((rc = check_ws(ws, ws_bytes, L)) != HMM_OK) return rc;
    unsigned char *w = (unsigned char *)ws;
    const int K = bank->K, N = bank->N, M = bank->M, S = batch->S, NP = viterbi_states(N);
    DevPtrs d = dev_ptrs(bank, batch, true);
    const int nbins = batch->max_len + 1;
    const TransposeJob tj{bank->B, (float *)(w + L.bt), N, M, NP, 1, nullptr};
    launch_plan(d, K, S, 1, batch->max_len, batch->total_symbols, nbins, w, L, stream, &tj);
    // ln A transposed: the same transpose with A's N columns in place of B's M
    launch_transpose(TransposeJob{bank->A, (float *)(w + L.lnat), N, N, NP, 1, nullptr}, K, stream);
    if (hipGetLastError() != hipSuccess) return HMM_ERR_HIP;
    VitLaunch v;
    memset(&v, 0, sizeof(v));
    v.K = K;
    v.N = N;
    v.M = M;
    v.NP = NP;
    v.S = S;
    v.max_len = batch->max_len;
    v.total = batch->total_symbols;
    v.perm = (const int32_t *)(w + L.perm);
    v.rowpos = (const int64_t *)(w + L.rowpos);
    v.rowsum = (int64_t *)(w + L.rowsum);
    v.state = (int32_t *)(w + L.queue);  // zeroed by the planner
    v.err = (int32_t *)(w + L.err);
    v.lnbt = (const float *)(w + L.bt);
    v.lnat = (const float *)(w + L.lnat);
    v.delta = (float *)(w + L.delta);
    v.spill = v.delta + (size_t)L.vit_rows * NP;
    v.score = score;
    v.path = path;
    v.cap_rows = L.vit_rows;
    const int cus = device_cu_count();
    v.max_grid = max_grid(L.wg_per_cu, cus);
    const int pr = prof_begin(stream, HMM_PROF_VITERBI);
    const hipError_t e = launch_viterbi(d, v, cus, stream);
    prof_end(stream, pr);
    return e == hipSuccess ? HMM_OK : HMM_ERR_HIP;
}

hmm_status hmm_plan_order(const hmm_bank *bank, const hmm_batch *batch, int32_t op, int32_t *order,
                          int32_t *group_start, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (op < HMM_OP_FORWARD || op > HMM_OP_VITERBI) return HMM_ERR_ARG;
    hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    if (batch->S > 0 && (!batch->offsets || !batch->lengths)) return HMM_ERR_NULL;
    if ((op == HMM_OP_GRAD || op == HMM_OP_VITERBI) && batch->S > 0 && !batch->model_of_seq) return HMM_ERR_NULL;
    if (!group_start || (batch->S > 0 && !order)) return HMM_ERR_NULL;
    const Layout L = make_layout(bank, batch, op);
    if ((rc = check_ws(ws, ws_bytes, L)) != HMM_OK) return rc;
    if (!batched_capable(bank, batch, op)) return HMM_ERR_UNSUPPORTED;
    const int groups = plan_groups(bank, batch, op);
    const bool own = groups > 1;
    DevPtrs d = dev_ptrs(bank, batch, own);
    unsigned char *w = (unsigned char *)ws;
    launch_plan(d, bank->K, batch->S, groups, batch->max_len, batch->total_symbols,
                groups * (batch->max_len + 1), w, L, stream);
    launch_copy_i32((const int32_t *)(w + L.perm), order, (size_t)batch->S, stream);
    launch_copy_i32((const int32_t *)(w + L.gstart), group_start, (size_t)groups + 1, stream);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_ERR_HIP;
}

hmm_status hmm_reestimate_rows(const float *n, const float *old, float *out, int64_t rows, int32_t cols,
                               hipStream_t stream) {
    if (rows < 0 || cols < 1) return HMM_ERR_SHAPE;
    if (rows > 0 && (!n || !old || !out)) return HMM_ERR_NULL;
    launch_reestimate_rows(n, old, out, rows, cols, stream);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_ERR_HIP;
}

hmm_status hmm_softmax_rows(const float *logits, float *probs, int64_t rows, int32_t cols, hipStream_t stream) {
    if (rows < 0 || cols < 1) return HMM_ERR_SHAPE;
    if (rows > 0 && (!logits || !probs)) return HMM_ERR_NULL;
    launch_softmax_rows(logits, probs, rows, cols, stream);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_ERR_HIP;
}

hmm_status hmm_logit_grad(const float *n, const float *probs, float *grad, int64_t rows, int32_t cols,
                          hipStream_t stream) {
    if (rows < 0 || cols < 1) return HMM_ERR_SHAPE;
    if (rows > 0 && (!n || !probs || !grad)) return HMM_ERR_NULL;
    launch_logit_grad(n, probs, grad, rows, cols, stream);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_ERR_HIP;
}

hmm_status hmm_workspace_error(const void *ws, hipStream_t stream, int32_t *first_bad_seq) {
    if (!ws || !first_bad_seq) return HMM_ERR_NULL;
    if (hipStreamSynchronize(stream) != hipSuccess) return HMM_ERR_HIP;
    int32_t v = INT32_MAX;
    if (hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return HMM_ERR_HIP;
    *first_bad_seq = (v == INT32_MAX) ? -1 : v;
    return HMM_OK;
}

hmm_status hmm_debug_flags(uint32_t *flags) {
    if (!flags) return HMM_ERR_NULL;
    *flags = 0;
#ifdef HMM_DEBUG
    if (hipDeviceSynchronize() != hipSuccess) return HMM_ERR_HIP;
    uint32_t (*const take[])() = {debug_take_planner, debug_take_fwd_plain, debug_take_fwd_mfma,
                                  debug_take_fwd_mfma32, debug_take_fwd_coop, debug_take_fwd_scan,
                                  debug_take_adj_mfma, debug_take_adj_coop, debug_take_viterbi,
                                  debug_take_abi};
    uint32_t v = 0;
    for (auto f : take) v |= f();
    if (v & 0x80000000u) return HMM_ERR_HIP;
    *flags = v;
    return HMM_OK;
#else
    return HMM_ERR_UNSUPPORTED;
#endif
}

hmm_status hmm_select_kernel(int32_t kind) {
    if (kind < HMM_KERNEL_AUTO || kind > HMM_KERNEL_SCAN) return HMM_ERR_ARG;
    g_kernel_kind.store(kind, std::memory_order_relaxed);
    return HMM_OK;
}

hmm_status hmm_call_kernel(const hmm_bank *bank, const hmm_batch *batch, int32_t op, int32_t *kernel) {
    if (!kernel) return HMM_ERR_NULL;
    if (op < HMM_OP_FORWARD || op > HMM_OP_VITERBI) return HMM_ERR_ARG;
    hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    const CallChoice cc = call_choice(bank, batch, op);
    if (op == HMM_OP_GRAD || op == HMM_OP_VITERBI) {
        if (!batched_capable(bank, batch, op)) return HMM_ERR_UNSUPPORTED;
        *kernel = op == HMM_OP_VITERBI ? HMM_KERNEL_BATCHED
                                       : (grad_uses_coop(padded_states(bank->N)) ? HMM_KERNEL_COOP : HMM_KERNEL_TILE16);
        return HMM_OK;
    }
    int fam = HMM_KERNEL_PLAIN;
    if ((rc = forward_family(bank, batch, op, cc.kind, &fam)) != HMM_OK) return rc;
    *kernel = fam;
    return HMM_OK;
}

hmm_status hmm_tune_key_of(const hmm_bank *bank, const hmm_batch *batch, int32_t op, hmm_tune_key *key) {
    if (!key) return HMM_ERR_NULL;
    if (op < HMM_OP_FORWARD || op > HMM_OP_VITERBI) return HMM_ERR_ARG;
    const hmm_status rc = check_shapes(bank, batch);
    if (rc != HMM_OK) return rc;
    *key = key_of(bank, batch, op);
    return HMM_OK;
}

static bool tune_key_valid(const hmm_tune_key *k) {
    return k->op >= HMM_OP_FORWARD && k->op <= HMM_OP_VITERBI && (k->all_pairs == 0 || k->all_pairs == 1) &&
           k->K >= 1 && k->K <= 65536 && k->N >= 1 && k->N <= HMM_MAX_STATES && k->M >= 1 &&
           k->M <= HMM_MAX_SYMBOLS && k->s_bucket >= 0 && k->s_bucket <= 31 && k->len_bucket >= 0 &&
           k->len_bucket <= 31;
}

hmm_status hmm_tune_set(const hmm_tune_key *key, const hmm_tune_choice *choice) {
    if (!key) return HMM_ERR_NULL;
    if (!tune_key_valid(key)) return HMM_ERR_ARG;
    if (choice) {
        if (choice->kernel < HMM_KERNEL_AUTO || choice->kernel > HMM_KERNEL_SCAN) return HMM_ERR_ARG;
        if ((key->op == HMM_OP_GRAD || key->op == HMM_OP_VITERBI) && choice->kernel != HMM_KERNEL_AUTO &&
            choice->kernel != HMM_KERNEL_BATCHED)
            return HMM_ERR_ARG;
        if (choice->wg_per_cu < 0 || choice->wg_per_cu > HMM_TUNE_MAX_WG) return HMM_ERR_ARG;
        if (choice->flags & ~(HMM_TUNE_XCD_OFF | HMM_TUNE_BT_GLOBAL | HMM_TUNE_BT_LDS)) return HMM_ERR_ARG;
        if ((choice->flags & HMM_TUNE_BT_GLOBAL) && (choice->flags & HMM_TUNE_BT_LDS)) return HMM_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int at = -1;
    for (int i = 0; i < g_tune_n; ++i)
        if (same_key(g_tune[i].key, *key)) at = i;
    if (!choice) {
        if (at >= 0) g_tune[at] = g_tune[--g_tune_n];
        return HMM_OK;
    }
    if (at < 0) {
        if (g_tune_n == HMM_TUNE_MAX) return HMM_ERR_UNSUPPORTED;
        at = g_tune_n++;
    }
    g_tune[at].key = *key;
    g_tune[at].choice = *choice;
    return HMM_OK;
}

hmm_status hmm_tune_get(const hmm_tune_key *key, hmm_tune_choice *choice, int32_t *found) {
    if (!key || !choice || !found) return HMM_ERR_NULL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *found = 0;
    for (int i = 0; i < g_tune_n; ++i)
        if (same_key(g_tune[i].key, *key)) {
            *choice = g_tune[i].choice;
            *found = 1;
            break;
        }
    return HMM_OK;
}

hmm_status hmm_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_n = 0;
    return HMM_OK;
}

hmm_status hmm_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    if (g_prof_on) g_prof_used = 0;
    return HMM_OK;
}

hmm_status hmm_profile_read(int32_t kernel, double *total_ms, int32_t *launches) {
    if (!total_ms || !launches) return HMM_ERR_NULL;
    if (kernel < HMM_PROF_FWD_BATCHED || kernel > HMM_PROF_VITERBI) return HMM_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double sum = 0.0;
    int n = 0;
    for (size_t i = 0; i < g_prof_used; ++i) {
        const ProfRecord &r = g_prof_pool[i];
        if (r.kind != kernel) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return HMM_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return HMM_ERR_HIP;
        sum += ms;
        ++n;
    }
    *total_ms = sum;
    *launches = n;
    return HMM_OK;
}

const char *hmm_status_string(int32_t s) {
    // an int, not the enum: any value may arrive through the C ABI
    switch (s) {
        case HMM_OK: return "HMM_OK";
        case HMM_ERR_NULL: return "HMM_ERR_NULL";
        case HMM_ERR_SHAPE: return "HMM_ERR_SHAPE";
        case HMM_ERR_WORKSPACE: return "HMM_ERR_WORKSPACE";
        case HMM_ERR_UNSUPPORTED: return "HMM_ERR_UNSUPPORTED";
        case HMM_ERR_HIP: return "HMM_ERR_HIP";
        case HMM_ERR_ARG: return "HMM_ERR_ARG";
    }
    return "HMM_ERR_UNKNOWN";
}

}  // extern "C"
