/*
 * Oracle (test infrastructure only): the learned-proposal sampler and the MLP
 * reference.  Neither is in the paper; they follow the project's reading.
 *
 * Buckets: b(v) = floor(log2(1 + deg(v))) clipped to [0, 31], from degrees.
 * Weights: an integer table w[j][b0][bp][bc] in [1, 2^16] per pattern, indexed
 * by the step j, the buckets of v_0 and v_{j-1} and the candidate's bucket.
 * Step j < k-1: S_j as in NS-prune; n_b = members of S_j in bucket b; Sigma =
 * sum_b n_b w_b; walking buckets in ascending b, the bucket is the first whose
 * running sum of n_b w_b exceeds floor(Sigma * r_j / 2^64); the member is the
 * floor(n_b * r_{16+j} / 2^64)-th member of that bucket in ascending id; the
 * weight factor is Sigma / w_b (one IEEE division).  The last step j = k-1
 * picks uniformly as NS-prune does (member floor(|S_j| * r_j / 2^64), factor
 * |S_j|): there every candidate completes exactly one match, so the uniform
 * pick is already the zero-variance choice.  alpha' = M times the factors in
 * step order (IEEE multiplications).  Any table with w >= 1 keeps the
 * estimator unbiased (importance sampling with full support).
 * Exact sums: X = alpha' * 2^52 is an integer for alpha' >= 1 (rejected when
 * alpha' >= 2^76), so the NS integer statistics apply unchanged; the predicted
 * error is scale invariant and the estimate is S1 / n / 2^52.
 *
 * MLP: s = w3 . relu(W2 relu(W1 x + b1) + b2) + b3, 16 -> 64 -> 64 -> 1, in
 * FP64 on BF16-rounded weights and inputs; loss = mean (s - y)^2 / 2.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

int32_t orc_bucket(const orc_graph* g, int64_t v) {
    int64_t d = g->off[v + 1] - g->off[v];
    int b = 0;
    while (b < 31 && ((d + 1) >> (b + 1)) > 0) b++;
    return b;
}

/* draws (nullable, 24 entries) overrides the Philox values draw d = draws[d]. */
void orc_ns_sample_learned(const orc_graph* g, const orc_plan* p, const uint16_t* table, uint64_t seed,
                           uint32_t tag, uint64_t s, const uint64_t* draws, orc_rec* r, double* alpha_f) {
    memset(r, 0, sizeof(*r));
    r->s = s;
    r->k = p->k;
    for (int i = 0; i < 8; i++) r->v[i] = -1;
    uint64_t M = p->oriented ? (uint64_t)g->m : 2 * (uint64_t)g->m;
    r->size[0] = M;
    *alpha_f = 0.0;
    if (M == 0) { r->fail_step = 1; return; }
#define DRAW(d) (draws ? draws[(d)] : orc_draw(seed, s, (uint32_t)(d), tag))
    uint64_t e = orc_mulhi(M, DRAW(0));
    if (p->oriented) { r->v[0] = g->esrc[e]; r->v[1] = g->edst[e]; }
    else { r->v[0] = g->arow[e]; r->v[1] = g->nbr[e]; }
    double a = (double)M;
    int32_t* buf = NULL;
    int b0 = orc_bucket(g, r->v[0]);
    for (int j = 2; j < p->k; j++) {
        uint64_t cnt = orc_candidates(g, p, j, r->v, NULL);
        r->size[j] = cnt;
        if (cnt == 0) { r->fail_step = j; free(buf); return; }
        buf = (int32_t*)realloc(buf, sizeof(int32_t) * (size_t)cnt);
        orc_candidates(g, p, j, r->v, buf);
        if (j == p->k - 1) {  /* last step: uniform pick */
            r->v[j] = buf[orc_mulhi(cnt, DRAW(j))];
            a = a * (double)cnt;
            continue;
        }
        int bp = orc_bucket(g, r->v[j - 1]);
        const uint16_t* w = table + ((((size_t)j * 32 + (size_t)b0) * 32 + (size_t)bp) * 32);
        uint64_t nb[32] = {0};
        for (uint64_t i = 0; i < cnt; i++) nb[orc_bucket(g, buf[i])]++;
        uint64_t sigma = 0;
        for (int b = 0; b < 32; b++) sigma += nb[b] * (uint64_t)w[b];
        uint64_t t = orc_mulhi(sigma, DRAW(j));
        uint64_t run = 0;
        int bsel = -1;
        for (int b = 0; b < 32; b++) {
            run += nb[b] * (uint64_t)w[b];
            if (run > t) { bsel = b; break; }
        }
        uint64_t idx = orc_mulhi(nb[bsel], DRAW(16 + j));
        uint64_t seen = 0;
        for (uint64_t i = 0; i < cnt; i++)
            if (orc_bucket(g, buf[i]) == bsel) {
                if (seen == idx) { r->v[j] = buf[i]; break; }
                seen++;
            }
        double factor = (double)sigma / (double)w[bsel];
        a = a * factor;
    }
    free(buf);
    r->hit = 1;
    *alpha_f = a;
    if (!(a < 0x1p76)) { r->overflow = 1; return; }
    int ex;
    double fr = frexp(a, &ex);               /* a = fr * 2^ex, fr in [0.5, 1) */
    uint64_t mant = (uint64_t)ldexp(fr, 53);  /* 53-bit integer mantissa */
    int shift = ex - 53 + 52;                 /* X = a * 2^52 = mant * 2^shift, shift >= 0 */
    unsigned __int128 x = (unsigned __int128)mant << shift;
    r->alpha_lo = (uint64_t)x;
    r->alpha_hi = (uint64_t)(x >> 64);
#undef DRAW
}

/* ------------------------------------------------------------------ MLP */
#define NIN 16
#define NH 64

static double bf16_round(double x) {
    /* round an FP32 value to BF16 (nearest, ties to even) */
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

double orc_bf16(double x) { return bf16_round(x); }

/* params layout (floats): W1[NIN*NH] (row-major in->out), b1[NH], W2[NH*NH], b2[NH], w3[NH], b3[1] */
int orc_mlp_nparams(void) { return NIN * NH + NH + NH * NH + NH + NH + 1; }

/* Forward (and, when grads != NULL, backward of loss = sum_i (s_i - y_i)^2 / (2N)).
 * Weights and inputs are rounded to BF16 first; everything else is FP64. */
#define RB(x) (bf16 ? bf16_round(x) : (double)(x))
/* bf16 = 0 evaluates the same network without any BF16 rounding (for
 * finite-difference checks of the derivative code). */
double orc_mlp(const float* params, const float* X, const float* y, int64_t N, int bf16, double* s_out,
               double* grads) {
    const float* W1 = params;
    const float* b1 = W1 + NIN * NH;
    const float* W2 = b1 + NH;
    const float* b2 = W2 + NH * NH;
    const float* w3 = b2 + NH;
    const float* b3 = w3 + NH;
    double* gW1 = grads;
    double* gb1 = grads ? gW1 + NIN * NH : NULL;
    double* gW2 = grads ? gb1 + NH : NULL;
    double* gb2 = grads ? gW2 + NH * NH : NULL;
    double* gw3 = grads ? gb2 + NH : NULL;
    double* gb3 = grads ? gw3 + NH : NULL;
    if (grads) memset(grads, 0, sizeof(double) * (size_t)orc_mlp_nparams());
    double loss = 0.0;
    for (int64_t r = 0; r < N; r++) {
        double x[NIN], z1[NH], h1[NH], z2[NH], h2[NH];
        for (int i = 0; i < NIN; i++) x[i] = RB(X[r * NIN + i]);
        for (int o = 0; o < NH; o++) {
            double a = b1[o];
            for (int i = 0; i < NIN; i++) a += x[i] * RB(W1[i * NH + o]);
            z1[o] = a;
            h1[o] = a > 0 ? a : 0;
        }
        /* the second layer consumes BF16 activations, like the MFMA kernels */
        double h1b[NH];
        for (int o = 0; o < NH; o++) h1b[o] = RB(h1[o]);
        for (int o = 0; o < NH; o++) {
            double a = b2[o];
            for (int i = 0; i < NH; i++) a += h1b[i] * RB(W2[i * NH + o]);
            z2[o] = a;
            h2[o] = a > 0 ? a : 0;
        }
        double s = b3[0];
        for (int i = 0; i < NH; i++) s += h2[i] * RB(w3[i]);
        if (s_out) s_out[r] = s;
        if (!y) continue;
        double d = s - (double)y[r];
        loss += 0.5 * d * d / (double)N;
        if (!grads) continue;
        double ds = d / (double)N;
        gb3[0] += ds;
        double dz2[NH];
        for (int i = 0; i < NH; i++) {
            gw3[i] += ds * h2[i];
            dz2[i] = z2[i] > 0 ? ds * RB(w3[i]) : 0.0;
            gb2[i] += dz2[i];
        }
        double dz1[NH];
        for (int i = 0; i < NH; i++) {
            double a = 0.0;
            for (int o = 0; o < NH; o++) {
                gW2[i * NH + o] += h1b[i] * dz2[o];
                a += RB(W2[i * NH + o]) * dz2[o];
            }
            dz1[i] = z1[i] > 0 ? a : 0.0;
            gb1[i] += dz1[i];
        }
        for (int i = 0; i < NIN; i++)
            for (int o = 0; o < NH; o++) gW1[i * NH + o] += x[i] * dz1[o];
    }
    return loss;
}

#undef RB

/* ------------------------------------------------------------------ table */
/* The learned proposal's weight table (a project extension; the paper's
 * lemma of Sec. 4.2 only asks for positive weights).  Cell (j, b0, bp, bc):
 * step j, degree buckets of v0, of v_{j-1} and of the candidate.  Its features
 * are, in order: bc/16, b0/16, bp/16, j/8, (bc-bp)/16, (bc-b0)/16, 1, the
 * one-hot pattern index (8 slots), 0; its score is the network on them.  The
 * 32 weights of a row (j, b0, bp) are 2^(score - row maximum + 15) rounded to
 * nearest and held in [1, 65535]; steps outside 2 .. k-2 hold 1 (step k-1, the
 * last, picks uniformly).  bf16 as in orc_mlp. */
void orc_learned_features(int pattern, int j, int b0, int bp, int bc, float* x) {
    x[0] = (float)bc / 16.f;
    x[1] = (float)b0 / 16.f;
    x[2] = (float)bp / 16.f;
    x[3] = (float)j / 8.f;
    x[4] = (float)(bc - bp) / 16.f;
    x[5] = (float)(bc - b0) / 16.f;
    x[6] = 1.f;
    for (int i = 0; i < 8; i++) x[7 + i] = i == pattern ? 1.f : 0.f;
    x[15] = 0.f;
}

void orc_learned_table(const float* params, int pattern, int k, int bf16, uint16_t* out) {
    float x[32 * NIN];
    double s[32];
    for (int j = 0; j < 8; j++)
        for (int b0 = 0; b0 < 32; b0++)
            for (int bp = 0; bp < 32; bp++) {
                uint16_t* row = out + (((size_t)j * 32 + (size_t)b0) * 32 + (size_t)bp) * 32;
                if (j < 2 || j > k - 2) {
                    for (int bc = 0; bc < 32; bc++) row[bc] = 1;
                    continue;
                }
                for (int bc = 0; bc < 32; bc++) orc_learned_features(pattern, j, b0, bp, bc, x + bc * NIN);
                orc_mlp(params, x, NULL, 32, bf16, s, NULL);
                double mx = s[0];
                for (int bc = 1; bc < 32; bc++)
                    if (s[bc] > mx) mx = s[bc];
                for (int bc = 0; bc < 32; bc++) {
                    double w = nearbyint(exp2(s[bc] - mx + 15.0));
                    if (w < 1.0) w = 1.0;
                    if (w > 65535.0) w = 65535.0;
                    row[bc] = (uint16_t)w;
                }
            }
}
