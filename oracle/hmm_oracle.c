/*
 * FP64 CPU oracle for the discrete-HMM bank (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header or table with
 * the GPU library.  It is deliberately plain: no blocking, no fusion, natural
 * index order, one sequence at a time (OpenMP only distributes whole
 * sequences or whole models over threads and never changes the arithmetic).
 *
 * Model (paper Sec. 2.7: activity recognition with one discrete HMM per
 * action; Sec. 3 item 3: the HMMs of the actions are evaluated independently).
 * The paper gives no formulas; the textbook discrete HMM is used:
 *   pi[i]     = P(q_1 = i)
 *   A[i][j]   = P(q_{t+1} = j | q_t = i)          (row-stochastic, alpha is a row vector)
 *   B[i][o]   = P(o_t = o | q_t = i)
 *   P(O | lambda) = sum over state paths of pi[q_1] B[q_1][o_1] prod_{t>=2} A[q_{t-1}][q_t] B[q_t][o_t].
 *
 * Scaled forward recursion (the "Forward" function of Sec. 2.7):
 *   alpha~_1(i) = pi[i] B[i][o_1]
 *   alpha~_t(j) = (sum_i alphahat_{t-1}(i) A[i][j]) B[j][o_t]      t >= 2
 *   c_t = sum_j alpha~_t(j),  alphahat_t = alpha~_t / c_t
 *   log P(O | lambda) = sum_t ln c_t.
 * T = 0 gives log P = 0.  A zero normaliser c_t gives -inf (impossible
 * observation).  A symbol outside [0, M) or a negative length gives NaN.
 *
 * Scaled backward recursion and expected counts (E-step of Baum-Welch, the
 * third function named in Sec. 2.7), with the same c_t:
 *   betahat_T(i) = 1
 *   w_{t+1}(j)   = B[j][o_{t+1}] betahat_{t+1}(j) / c_{t+1}
 *   betahat_t(i) = sum_j A[i][j] w_{t+1}(j)
 *   gamma_t(i)   = alphahat_t(i) betahat_t(i)
 *   xi_t(i,j)    = alphahat_t(i) A[i][j] w_{t+1}(j)
 *   n_pi[i]   += w_s gamma_1(i)
 *   n_A[i][j] += w_s sum_{t<T} xi_t(i,j)
 *   n_B[i][o] += w_s sum_{t: o_t = o} gamma_t(i)
 * where w_s is the weight of sequence s.  These counts are the gradient of
 * sum_s w_s log P(O_s | lambda_{m(s)}) with respect to ln pi, ln A and ln B.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int seq_is_valid(int M, const int32_t *o, int32_t T) {
    if (T < 0) return 0;
    for (int32_t t = 0; t < T; ++t)
        if (o[t] < 0 || o[t] >= M) return 0;
    return 1;
}

/* log P(O | lambda) of one sequence under one model. */
static double forward_one(int N, int M, const double *pi, const double *A, const double *B,
                          const int32_t *o, int32_t T, double *ahat, double *atil) {
    if (!seq_is_valid(M, o, T)) return NAN;
    if (T == 0) return 0.0;
    double loglik = 0.0;
    for (int t = 0; t < T; ++t) {
        if (t == 0) {
            for (int i = 0; i < N; ++i) atil[i] = pi[i] * B[(size_t)i * M + o[0]];
        } else {
            for (int j = 0; j < N; ++j) {
                double u = 0.0;
                for (int i = 0; i < N; ++i) u += ahat[i] * A[(size_t)i * N + j];
                atil[j] = u * B[(size_t)j * M + o[t]];
            }
        }
        double c = 0.0;
        for (int i = 0; i < N; ++i) c += atil[i];
        if (!(c > 0.0)) {
            if (c == 0.0) return -INFINITY;
            return NAN;
        }
        for (int i = 0; i < N; ++i) ahat[i] = atil[i] / c;
        loglik += log(c);
    }
    return loglik;
}

/*
 * Log-likelihoods.
 *   model_of_seq == NULL: every sequence against every model, out[s*K + k].
 *   otherwise:            sequence s against model model_of_seq[s], out[s].
 * Returns 0, or -1 on bad arguments (a model index outside [0, K)).
 */
int oracle_forward(int K, int N, int M, const double *pi, const double *A, const double *B,
                   int S, const int32_t *symbols, const int64_t *offsets, const int32_t *lengths,
                   const int32_t *model_of_seq, double *out, int nthreads) {
    if (K <= 0 || N <= 0 || M <= 0 || S < 0) return -1;
    if (model_of_seq)
        for (int s = 0; s < S; ++s)
            if (model_of_seq[s] < 0 || model_of_seq[s] >= K) return -1;
    const int64_t npairs = model_of_seq ? (int64_t)S : (int64_t)S * K;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *ahat = (double *)malloc(sizeof(double) * (size_t)N);
        double *atil = (double *)malloc(sizeof(double) * (size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npairs; ++p) {
            int s = model_of_seq ? (int)p : (int)(p / K);
            int k = model_of_seq ? model_of_seq[s] : (int)(p % K);
            const double *pk = pi + (size_t)k * N;
            const double *Ak = A + (size_t)k * N * N;
            const double *Bk = B + (size_t)k * N * M;
            out[p] = forward_one(N, M, pk, Ak, Bk, symbols + offsets[s], lengths[s], ahat, atil);
        }
        free(ahat);
        free(atil);
    }
    return 0;
}

/*
 * Recognition: label[s] = smallest k attaining max_k loglik[s][k]; NaN entries
 * are skipped; a row of only NaN gives -1.  -inf is an ordinary value.
 */
void oracle_classify(int S, int K, const double *loglik, int32_t *labels) {
    for (int s = 0; s < S; ++s) {
        int best = -1;
        double bv = 0.0;
        for (int k = 0; k < K; ++k) {
            double v = loglik[(size_t)s * K + k];
            if (isnan(v)) continue;
            if (best < 0 || v > bv) {
                best = k;
                bv = v;
            }
        }
        labels[s] = best;
    }
}

/* Same decision taken on FP32 values (the precision the GPU decides in). */
void oracle_classify_f32(int S, int K, const float *loglik, int32_t *labels) {
    for (int s = 0; s < S; ++s) {
        int best = -1;
        float bv = 0.0f;
        for (int k = 0; k < K; ++k) {
            float v = loglik[(size_t)s * K + k];
            if (isnan(v)) continue;
            if (best < 0 || v > bv) {
                best = k;
                bv = v;
            }
        }
        labels[s] = best;
    }
}

/*
 * Full scaled forward / backward trace of one sequence (for invariant checks).
 * ahat[T][N], bhat[T][N], c[T].  Returns log P, as forward_one.
 */
double oracle_trace(int N, int M, const double *pi, const double *A, const double *B,
                    const int32_t *o, int32_t T, double *ahat, double *bhat, double *c) {
    if (!seq_is_valid(M, o, T)) return NAN;
    if (T == 0) return 0.0;
    double loglik = 0.0;
    int dead = 0;
    for (int t = 0; t < T; ++t) {
        double *at = ahat + (size_t)t * N;
        if (t == 0) {
            for (int i = 0; i < N; ++i) at[i] = pi[i] * B[(size_t)i * M + o[0]];
        } else {
            const double *ap = ahat + (size_t)(t - 1) * N;
            for (int j = 0; j < N; ++j) {
                double u = 0.0;
                for (int i = 0; i < N; ++i) u += ap[i] * A[(size_t)i * N + j];
                at[j] = u * B[(size_t)j * M + o[t]];
            }
        }
        double ct = 0.0;
        for (int i = 0; i < N; ++i) ct += at[i];
        c[t] = ct;
        if (!(ct > 0.0)) {
            dead = 1;
            break;
        }
        for (int i = 0; i < N; ++i) at[i] /= ct;
        loglik += log(ct);
    }
    if (dead) return -INFINITY;
    for (int i = 0; i < N; ++i) bhat[(size_t)(T - 1) * N + i] = 1.0;
    for (int t = T - 2; t >= 0; --t) {
        const double *bn = bhat + (size_t)(t + 1) * N;
        double *bt = bhat + (size_t)t * N;
        for (int i = 0; i < N; ++i) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j)
                acc += A[(size_t)i * N + j] * (B[(size_t)j * M + o[t + 1]] * bn[j] / c[t + 1]);
            bt[i] = acc;
        }
    }
    return loglik;
}

/*
 * Expected counts (gradient of sum_s w_s log P w.r.t. the log-parameters) for
 * each sequence paired with its own model.  weights == NULL means all ones.
 * loglik[S] receives log P of each pair.  Counts are overwritten.  Sequences
 * with an invalid symbol or length get NaN log-likelihood and add nothing;
 * impossible sequences (-inf) add nothing.
 * Models are distributed over threads; each model's sequences are visited in
 * index order, so the result does not depend on the thread count.
 */
int oracle_counts(int K, int N, int M, const double *pi, const double *A, const double *B,
                  int S, const int32_t *symbols, const int64_t *offsets, const int32_t *lengths,
                  const int32_t *model_of_seq, const double *weights, double *loglik,
                  double *cnt_pi, double *cnt_A, double *cnt_B, int nthreads) {
    if (K <= 0 || N <= 0 || M <= 0 || S < 0 || !model_of_seq) return -1;
    for (int s = 0; s < S; ++s)
        if (model_of_seq[s] < 0 || model_of_seq[s] >= K) return -1;
    memset(cnt_pi, 0, sizeof(double) * (size_t)K * N);
    memset(cnt_A, 0, sizeof(double) * (size_t)K * N * N);
    memset(cnt_B, 0, sizeof(double) * (size_t)K * N * M);
    int32_t Tmax = 0;
    for (int s = 0; s < S; ++s)
        if (lengths[s] > Tmax) Tmax = lengths[s];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        size_t Tc = Tmax > 0 ? (size_t)Tmax : 1;
        double *ahat = (double *)malloc(sizeof(double) * Tc * N);
        double *bhat = (double *)malloc(sizeof(double) * Tc * N);
        double *c = (double *)malloc(sizeof(double) * Tc);
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < K; ++k) {
            const double *pk = pi + (size_t)k * N;
            const double *Ak = A + (size_t)k * N * N;
            const double *Bk = B + (size_t)k * N * M;
            double *npi = cnt_pi + (size_t)k * N;
            double *nA = cnt_A + (size_t)k * N * N;
            double *nB = cnt_B + (size_t)k * N * M;
            for (int s = 0; s < S; ++s) {
                if (model_of_seq[s] != k) continue;
                const int32_t *o = symbols + offsets[s];
                int32_t T = lengths[s];
                double ws = weights ? weights[s] : 1.0;
                double ll = oracle_trace(N, M, pk, Ak, Bk, o, T, ahat, bhat, c);
                loglik[s] = ll;
                if (!isfinite(ll) || T == 0) continue;
                for (int t = 0; t < T; ++t) {
                    const double *at = ahat + (size_t)t * N;
                    const double *bt = bhat + (size_t)t * N;
                    for (int i = 0; i < N; ++i) {
                        double g = at[i] * bt[i];
                        if (t == 0) npi[i] += ws * g;
                        nB[(size_t)i * M + o[t]] += ws * g;
                    }
                    if (t + 1 < T) {
                        const double *bn = bhat + (size_t)(t + 1) * N;
                        for (int i = 0; i < N; ++i)
                            for (int j = 0; j < N; ++j) {
                                double w = Bk[(size_t)j * M + o[t + 1]] * bn[j] / c[t + 1];
                                nA[(size_t)i * N + j] += ws * at[i] * Ak[(size_t)i * N + j] * w;
                            }
                    }
                }
            }
        }
        free(ahat);
        free(bhat);
        free(c);
    }
    return 0;
}

/*
 * Most likely state path (the "Viterbi" function of Sec. 2.7), in the log
 * domain, each sequence with its own model:
 *   delta_1(i) = ln pi[i] + ln B[i][o_1]
 *   delta_t(j) = max_i (delta_{t-1}(i) + ln A[i][j]) + ln B[j][o_t]        t >= 2
 *   psi_t(j)   = the smallest i attaining that maximum
 *   score      = max_j delta_T(j);  q_T = the smallest j attaining it;  q_{t-1} = psi_t(q_t)
 * with ln 0 = -inf ("attaining" compares exactly, so when every candidate is
 * -inf the smallest index is taken).  T = 0 gives score 0 and an empty path;
 * an invalid symbol or length gives score NaN and a path of -1.
 * margin[s] (may be NULL) receives the smallest gap, over the final choice and
 * every backtracking choice on the returned path, between the chosen
 * candidate and the best other candidate (+inf when N = 1 or T = 0): when it is
 * large compared with the rounding of an implementation, that implementation
 * must return the same path.
 */
int oracle_viterbi(int K, int N, int M, const double *pi, const double *A, const double *B, int S,
                   const int32_t *symbols, const int64_t *offsets, const int32_t *lengths,
                   const int32_t *model_of_seq, double *score, int32_t *path, double *margin, int nthreads) {
    if (K <= 0 || N <= 0 || M <= 0 || S < 0 || !model_of_seq) return -1;
    for (int s = 0; s < S; ++s)
        if (model_of_seq[s] < 0 || model_of_seq[s] >= K) return -1;
    int32_t Tmax = 0;
    for (int s = 0; s < S; ++s)
        if (lengths[s] > Tmax) Tmax = lengths[s];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        size_t Tc = Tmax > 0 ? (size_t)Tmax : 1;
        double *delta = (double *)malloc(sizeof(double) * Tc * N);
        int32_t *psi = (int32_t *)malloc(sizeof(int32_t) * Tc * N);
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < S; ++s) {
            const int k = model_of_seq[s];
            const double *pk = pi + (size_t)k * N;
            const double *Ak = A + (size_t)k * N * N;
            const double *Bk = B + (size_t)k * N * M;
            const int32_t *o = symbols + offsets[s];
            const int32_t T = lengths[s];
            int32_t *q = path + offsets[s];
            if (!seq_is_valid(M, o, T)) {
                score[s] = NAN;
                for (int32_t t = 0; t < T; ++t) q[t] = -1;
                if (margin) margin[s] = NAN;
                continue;
            }
            if (T == 0) {
                score[s] = 0.0;
                if (margin) margin[s] = INFINITY;
                continue;
            }
            for (int i = 0; i < N; ++i) delta[i] = log(pk[i]) + log(Bk[(size_t)i * M + o[0]]);
            for (int t = 1; t < T; ++t) {
                const double *dp = delta + (size_t)(t - 1) * N;
                double *dt = delta + (size_t)t * N;
                for (int j = 0; j < N; ++j) {
                    double best = -INFINITY;
                    int arg = 0;
                    for (int i = 0; i < N; ++i) {
                        const double cand = dp[i] + log(Ak[(size_t)i * N + j]);
                        if (cand > best) {
                            best = cand;
                            arg = i;
                        }
                    }
                    dt[j] = best + log(Bk[(size_t)j * M + o[t]]);
                    psi[(size_t)t * N + j] = arg;
                }
            }
            const double *dl = delta + (size_t)(T - 1) * N;
            double best = -INFINITY;
            int arg = 0;
            for (int j = 0; j < N; ++j)
                if (dl[j] > best) {
                    best = dl[j];
                    arg = j;
                }
            score[s] = best;
            q[T - 1] = arg;
            for (int32_t t = T - 1; t > 0; --t) q[t - 1] = psi[(size_t)t * N + q[t]];
            if (margin) {
                /* gap between the chosen candidate and the best other one, at each choice */
                double gap = INFINITY;
                for (int j = 0; j < N; ++j)
                    if (j != q[T - 1] && best - dl[j] < gap) gap = best - dl[j];
                for (int32_t t = T - 1; t > 0; --t) {
                    const double *dp = delta + (size_t)(t - 1) * N;
                    const int j = q[t], c = q[t - 1];
                    const double chosen = dp[c] + log(Ak[(size_t)c * N + j]);
                    for (int i = 0; i < N; ++i) {
                        if (i == c) continue;
                        const double g = chosen - (dp[i] + log(Ak[(size_t)i * N + j]));
                        if (g < gap) gap = g;
                    }
                }
                margin[s] = gap;
            }
        }
        free(delta);
        free(psi);
    }
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
