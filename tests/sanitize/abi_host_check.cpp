// Host-side paths of libhmm_mi355x under AddressSanitizer and UndefinedBehaviorSanitizer
// (built and run by tests/test_sanitizers.py on a machine without a GPU).  Every call
// below returns before anything would be enqueued: workspace sizing over a grid of
// shapes, the argument checks of every entry point, the tuning table (filled to
// capacity, replaced, removed, cleared), call-shape keys and kernel resolution,
// profiling records, and status strings.  Exit status 0 when every expectation holds.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "hmm.h"

static int failures = 0;
#define EXPECT(cond)                                                       \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static const float *F(uintptr_t p) { return reinterpret_cast<const float *>(p); }

static hmm_bank bank(int K, int N, int M) { return hmm_bank{K, N, M, F(0x1000), F(0x2000), F(0x3000)}; }

static hmm_batch batch(int S, int max_len, int64_t total, bool models) {
    return hmm_batch{S, reinterpret_cast<const int32_t *>(0x4000), reinterpret_cast<const int64_t *>(0x5000),
                     reinterpret_cast<const int32_t *>(0x6000),
                     models ? reinterpret_cast<const int32_t *>(0x7000) : nullptr, max_len, total};
}

static void workspace_grid() {
    const int Ks[] = {1, 3, 64, 65536};
    const int Ns[] = {1, 5, 16, 17, 33, 48, 64, 65, 100, 128, 129, 200, 256};
    const int Ms[] = {1, 7, 256, 1024};
    const int Ss[] = {0, 1, 100, 65536};
    const int Ls[] = {0, 1, 64, 2048, 4096};
    for (int K : Ks)
        for (int N : Ns)
            for (int M : Ms)
                for (int S : Ss)
                    for (int L : Ls)
                        for (int models = 0; models < 2; ++models)
                            for (int op = HMM_OP_FORWARD; op <= HMM_OP_VITERBI; ++op) {
                                const hmm_bank b = bank(K, N, M);
                                const hmm_batch q = batch(S, L, (int64_t)S * L, models != 0);
                                const size_t n = hmm_workspace_size(&b, &q, op);
                                EXPECT(n > 0);
                                int32_t kern = -1;
                                const hmm_status rc = hmm_call_kernel(&b, &q, op, &kern);
                                EXPECT(rc == HMM_OK || rc == HMM_ERR_UNSUPPORTED);
                                hmm_tune_key key;
                                EXPECT(hmm_tune_key_of(&b, &q, op, &key) == HMM_OK);
                                if (op == HMM_OP_VITERBI) {
                                    // the least and the most rows a round may keep
                                    const int64_t lo = 2 * (int64_t)L < q.total_symbols ? 2 * (int64_t)L : q.total_symbols;
                                    const size_t a = hmm_viterbi_workspace_size(&b, &q, lo);
                                    const size_t z = hmm_viterbi_workspace_size(&b, &q, INT64_MAX);
                                    EXPECT(a > 0 && a <= n && n <= z);
                                    EXPECT(lo == 0 || hmm_viterbi_workspace_size(&b, &q, lo - 1) == 0);
                                }
                                if (op == HMM_OP_GRAD) {
                                    // checkpoints only, the default, and every step of S max_len rows
                                    const size_t c = hmm_grad_workspace_size(&b, &q, 0);
                                    const size_t f = hmm_grad_workspace_size(&b, &q, INT64_MAX);
                                    EXPECT(c > 0 && c <= n && n <= f);
                                    EXPECT(hmm_grad_workspace_size(&b, &q, (int64_t)S * L) == f);
                                    EXPECT(hmm_grad_workspace_size(&b, &q, -1) == 0);
                                }
                            }
    // out-of-range shapes size nothing
    const hmm_batch q = batch(100, 50, 5000, false);
    hmm_bank bad = bank(0, 16, 32);
    EXPECT(hmm_workspace_size(&bad, &q, 0) == 0);
    bad = bank(4, 257, 32);
    EXPECT(hmm_workspace_size(&bad, &q, 0) == 0);
    bad = bank(4, 16, HMM_MAX_SYMBOLS + 1);
    EXPECT(hmm_workspace_size(&bad, &q, 0) == 0);
    const hmm_bank b = bank(4, 16, 32);
    hmm_batch big = batch(100, HMM_MAX_LEN + 1, 5000, false);
    EXPECT(hmm_workspace_size(&b, &big, 0) == 0);
    big = batch(-1, 50, 5000, false);
    EXPECT(hmm_workspace_size(&b, &big, 0) == 0);
    EXPECT(hmm_workspace_size(&b, &q, 7) == 0);
    EXPECT(hmm_workspace_size(nullptr, &q, 0) == 0);
    EXPECT(hmm_workspace_size(&b, nullptr, 0) == 0);
}

static void argument_checks() {
    const hmm_bank b = bank(4, 16, 32);
    const hmm_batch q = batch(100, 50, 5000, false);
    const hmm_batch qm = batch(100, 50, 5000, true);
    float *out = reinterpret_cast<float *>(0x8000);
    int32_t *lab = reinterpret_cast<int32_t *>(0x9000);
    void *ws = reinterpret_cast<void *>(0x100000);
    EXPECT(hmm_forward_loglik(nullptr, &q, out, ws, 1ull << 30, nullptr) == HMM_ERR_NULL);
    hmm_bank nb = b;
    nb.A = nullptr;
    EXPECT(hmm_forward_loglik(&nb, &q, out, ws, 1ull << 30, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_forward_loglik(&b, &q, nullptr, ws, 1ull << 30, nullptr) == HMM_ERR_NULL);
    const size_t need = hmm_workspace_size(&b, &q, HMM_OP_FORWARD);
    EXPECT(hmm_forward_loglik(&b, &q, out, ws, need - 1, nullptr) == HMM_ERR_WORKSPACE);
    EXPECT(hmm_forward_loglik(&b, &q, out, nullptr, need, nullptr) == HMM_ERR_WORKSPACE);
    EXPECT(hmm_forward_loglik(&b, &q, out, reinterpret_cast<void *>(0x100004), need, nullptr) == HMM_ERR_WORKSPACE);
    EXPECT(hmm_classify(&b, &q, nullptr, nullptr, ws, 1ull << 30, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_classify(&b, &q, lab, nullptr, ws, 16, nullptr) == HMM_ERR_WORKSPACE);
    // the static-scratch variant refuses a batch beyond its array before touching the device
    const hmm_bank c3 = bank(64, 32, 256);
    const hmm_batch huge = batch(200000, 2048, 200000ll * 1000, false);
    EXPECT(hmm_classify_noalloc(&c3, &huge, lab, nullptr, nullptr) == HMM_ERR_WORKSPACE);
    EXPECT(hmm_classify_noalloc(nullptr, &huge, lab, nullptr, nullptr) == HMM_ERR_NULL);
    // gradient: model_of_seq, counts and the phase
    EXPECT(hmm_forward_backward_grad(&b, &q, nullptr, out, out, out, out, 0, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_forward_backward_grad(&b, &qm, nullptr, out, nullptr, out, out, 0, ws, 1ull << 40, nullptr) ==
           HMM_ERR_NULL);
    EXPECT(hmm_forward_backward_grad(&b, &qm, nullptr, out, out, out, out, 3, ws, 1ull << 40, nullptr) == HMM_ERR_ARG);
    EXPECT(hmm_forward_backward_grad(&b, &qm, nullptr, out, out, out, out, 0, ws, 16, nullptr) == HMM_ERR_WORKSPACE);
    const hmm_bank wide = bank(64, 16, 32);
    const hmm_batch longq = batch(100, 1 << 20, 5000, true);
    const size_t gneed = hmm_workspace_size(&wide, &longq, HMM_OP_GRAD);
    EXPECT(hmm_forward_backward_grad(&wide, &longq, nullptr, out, out, out, out, 0, ws, gneed, nullptr) ==
           HMM_ERR_UNSUPPORTED);
    // Viterbi
    EXPECT(hmm_viterbi(&b, &q, out, lab, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_viterbi(&b, &qm, nullptr, lab, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_viterbi(&b, &qm, out, nullptr, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    const size_t vleast = hmm_viterbi_workspace_size(&b, &qm, 100);
    EXPECT(vleast > 0 && vleast <= hmm_workspace_size(&b, &qm, HMM_OP_VITERBI));
    EXPECT(hmm_viterbi(&b, &qm, out, lab, ws, vleast - 1, nullptr) == HMM_ERR_WORKSPACE);
    EXPECT(hmm_viterbi(&b, &qm, out, lab, nullptr, 1ull << 40, nullptr) == HMM_ERR_WORKSPACE);
    EXPECT(hmm_viterbi_workspace_size(&b, &qm, 99) == 0);
    EXPECT(hmm_viterbi_workspace_size(nullptr, &qm, 100) == 0);
    // work list: operation range, model_of_seq for own-model operations, outputs, workspace
    int32_t *ord = reinterpret_cast<int32_t *>(0xa000);
    EXPECT(hmm_plan_order(&b, &qm, 4, ord, lab, ws, 1ull << 40, nullptr) == HMM_ERR_ARG);
    EXPECT(hmm_plan_order(&b, &qm, -1, ord, lab, ws, 1ull << 40, nullptr) == HMM_ERR_ARG);
    EXPECT(hmm_plan_order(&b, &q, HMM_OP_GRAD, ord, lab, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_plan_order(&b, &q, HMM_OP_VITERBI, ord, lab, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_plan_order(&b, &qm, HMM_OP_FORWARD, nullptr, lab, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_plan_order(&b, &qm, HMM_OP_FORWARD, ord, nullptr, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_plan_order(&b, &qm, HMM_OP_FORWARD, ord, lab, ws, 16, nullptr) == HMM_ERR_WORKSPACE);
    EXPECT(hmm_plan_order(nullptr, &qm, HMM_OP_FORWARD, ord, lab, ws, 1ull << 40, nullptr) == HMM_ERR_NULL);
    // row kernels
    EXPECT(hmm_reestimate_rows(out, out, out, -1, 4, nullptr) == HMM_ERR_SHAPE);
    EXPECT(hmm_reestimate_rows(nullptr, out, out, 3, 4, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_softmax_rows(out, out, -1, 4, nullptr) == HMM_ERR_SHAPE);
    EXPECT(hmm_softmax_rows(nullptr, out, 4, 4, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_logit_grad(out, out, out, 4, 0, nullptr) == HMM_ERR_SHAPE);
    EXPECT(hmm_logit_grad(out, nullptr, out, 4, 4, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_workspace_error(nullptr, nullptr, nullptr) == HMM_ERR_NULL);
    uint32_t dbg = 5;
    EXPECT(hmm_debug_flags(nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_debug_flags(&dbg) == HMM_ERR_UNSUPPORTED && dbg == 0);  // normal build: no checks
    EXPECT(hmm_select_kernel(7) == HMM_ERR_ARG);
    EXPECT(hmm_select_kernel(-1) == HMM_ERR_ARG);
    for (int k = HMM_KERNEL_SCAN; k >= HMM_KERNEL_AUTO; --k) EXPECT(hmm_select_kernel(k) == HMM_OK);
}

static hmm_tune_key key(int op, int all_pairs, int K, int N, int M, int sb, int lb) {
    hmm_tune_key k;
    std::memset(&k, 0, sizeof(k));
    k.op = op;
    k.all_pairs = all_pairs;
    k.K = K;
    k.N = N;
    k.M = M;
    k.s_bucket = sb;
    k.len_bucket = lb;
    return k;
}

static void tuning_table() {
    EXPECT(hmm_tune_clear() == HMM_OK);
    const hmm_tune_choice c16{HMM_KERNEL_TILE16, 1, 0}, c32{HMM_KERNEL_TILE32, 2, HMM_TUNE_XCD_OFF | HMM_TUNE_BT_LDS};
    for (int i = 0; i < HMM_TUNE_MAX; ++i) {
        const hmm_tune_key k = key(HMM_OP_FORWARD, 1, i + 1, 16, 32, 7, 6);
        EXPECT(hmm_tune_set(&k, &c16) == HMM_OK);
    }
    hmm_tune_key over = key(HMM_OP_FORWARD, 1, HMM_TUNE_MAX + 1, 16, 32, 7, 6);
    EXPECT(hmm_tune_set(&over, &c16) == HMM_ERR_UNSUPPORTED);
    const hmm_tune_key k5 = key(HMM_OP_FORWARD, 1, 5, 16, 32, 7, 6);
    EXPECT(hmm_tune_set(&k5, &c32) == HMM_OK);
    hmm_tune_choice got{0, 0, 0};
    int32_t found = 0;
    EXPECT(hmm_tune_get(&k5, &got, &found) == HMM_OK && found == 1 && got.kernel == HMM_KERNEL_TILE32 &&
           got.wg_per_cu == 2 && got.flags == (HMM_TUNE_XCD_OFF | HMM_TUNE_BT_LDS));
    const hmm_tune_key k7 = key(HMM_OP_FORWARD, 1, 7, 16, 32, 7, 6);
    EXPECT(hmm_tune_set(&k7, nullptr) == HMM_OK);
    EXPECT(hmm_tune_set(&over, &c16) == HMM_OK);
    EXPECT(hmm_tune_get(&k7, &got, &found) == HMM_OK && found == 0);
    // invalid keys and choices
    const hmm_tune_key bad_op = key(4, 1, 4, 16, 32, 7, 6), bad_pairs = key(0, 2, 4, 16, 32, 7, 6),
                       bad_n = key(0, 1, 4, 257, 32, 7, 6), bad_sb = key(0, 1, 4, 16, 32, 32, 6);
    EXPECT(hmm_tune_set(&bad_op, &c16) == HMM_ERR_ARG);
    EXPECT(hmm_tune_set(&bad_pairs, &c16) == HMM_ERR_ARG);
    EXPECT(hmm_tune_set(&bad_n, &c16) == HMM_ERR_ARG);
    EXPECT(hmm_tune_set(&bad_sb, &c16) == HMM_ERR_ARG);
    const hmm_tune_choice bad_kind{7, 0, 0}, bad_cap{HMM_KERNEL_AUTO, HMM_TUNE_MAX_WG + 1, 0};
    const hmm_tune_choice bad_bit{HMM_KERNEL_AUTO, 0, 8}, bad_pair{HMM_KERNEL_AUTO, 0, HMM_TUNE_BT_GLOBAL | HMM_TUNE_BT_LDS};
    EXPECT(hmm_tune_set(&k5, &bad_kind) == HMM_ERR_ARG);
    EXPECT(hmm_tune_set(&k5, &bad_cap) == HMM_ERR_ARG);
    EXPECT(hmm_tune_set(&k5, &bad_bit) == HMM_ERR_ARG);
    EXPECT(hmm_tune_set(&k5, &bad_pair) == HMM_ERR_ARG);
    const hmm_tune_key kg = key(HMM_OP_GRAD, 0, 8, 64, 512, 14, 10);
    EXPECT(hmm_tune_set(&kg, &c16) == HMM_ERR_ARG);
    EXPECT(hmm_tune_set(nullptr, nullptr) == HMM_ERR_NULL);
    EXPECT(hmm_tune_get(&k5, nullptr, nullptr) == HMM_ERR_NULL);
    // a table entry takes effect in sizing and resolution
    EXPECT(hmm_tune_clear() == HMM_OK);
    const hmm_bank b = bank(4, 16, 32);
    const hmm_batch q = batch(1000, 1000, 1000000, false);
    const size_t plain = hmm_workspace_size(&b, &q, HMM_OP_FORWARD);
    hmm_tune_key kq;
    EXPECT(hmm_tune_key_of(&b, &q, HMM_OP_FORWARD, &kq) == HMM_OK);
    const hmm_tune_choice scan{HMM_KERNEL_SCAN, 0, 0};
    EXPECT(hmm_tune_set(&kq, &scan) == HMM_OK);
    EXPECT(hmm_workspace_size(&b, &q, HMM_OP_FORWARD) > plain);
    int32_t kern = -1;
    EXPECT(hmm_call_kernel(&b, &q, HMM_OP_FORWARD, &kern) == HMM_OK && kern == HMM_KERNEL_SCAN);
    EXPECT(hmm_tune_clear() == HMM_OK);
    EXPECT(hmm_workspace_size(&b, &q, HMM_OP_FORWARD) == plain);
}

static void profiling_and_strings() {
    EXPECT(hmm_profile_enable(1) == HMM_OK);
    double ms = -1.0;
    int32_t n = -1;
    EXPECT(hmm_profile_read(HMM_PROF_FWD_BATCHED, &ms, &n) == HMM_OK && n == 0 && ms == 0.0);
    EXPECT(hmm_profile_read(9, &ms, &n) == HMM_ERR_ARG);
    EXPECT(hmm_profile_read(HMM_PROF_VITERBI, nullptr, &n) == HMM_ERR_NULL);
    EXPECT(hmm_profile_enable(0) == HMM_OK);
    const hmm_status all[] = {HMM_OK, HMM_ERR_NULL, HMM_ERR_SHAPE, HMM_ERR_WORKSPACE, HMM_ERR_UNSUPPORTED,
                              HMM_ERR_HIP, HMM_ERR_ARG};
    for (hmm_status s : all) EXPECT(std::strncmp(hmm_status_string((int32_t)s), "HMM_", 4) == 0);
    EXPECT(std::strcmp(hmm_status_string(42), "HMM_ERR_UNKNOWN") == 0);
}

int main() {
    workspace_grid();
    argument_checks();
    tuning_table();
    profiling_and_strings();
    if (failures) {
        std::fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    std::printf("abi host checks passed\n");
    return 0;
}
