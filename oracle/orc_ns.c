/*
 * Oracle (test infrastructure only): NS-prune sampler, online statistics and
 * the convergence rule.
 *
 * Sampler (Sec. 4.2, the 4-cycle NS-prune algorithm and the unbiasedness
 * lemma): draw the first edge uniformly (alpha = M, M = m oriented edges or
 * 2m arcs); for each later position j form the candidate set S_j = common
 * neighbours of the earlier positions joined to j by a pattern edge, minus (for
 * vertex-induced counting) neighbours of earlier positions not joined to j,
 * minus the earlier vertices, inside the symmetry-breaking bounds; an empty
 * S_j ends the sample as a miss (X = 0); otherwise pick one member uniformly and
 * multiply alpha by |S_j|.  A sample that reaches the last position is a hit
 * with X = alpha = M * prod |S_j|; no closure check is needed.
 *
 * Random numbers: draw d of sample s is Philox4x32-10 with key = seed and
 * counter = (s mod 2^32, s div 2^32, d, tag), taken as w1*2^32 + w0; the index
 * into a set of size N is floor(N * r / 2^64) applied to the ascending list.
 *
 * Statistics (Sec. 4.1, the NS-online algorithm and the error equation):
 * exact integers n, sum X, sum X^2; at each window end mu = S1/n and
 * eps_hat = z * sqrt((n*S2 - S1^2)/n) / S1 with z = Phi^-1(1 - delta/2), which
 * is the paper's z*sigma/mu with var = S2/n - mu^2 and sigma = sqrt(var/n)
 * rearranged so the subtraction is exact.  eps_hat = +inf while S1 = 0.
 * Stop at the first window end with eps_hat <= eps.
 */
#include "oracle.h"
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ big integers */
#define OB 24 /* 32-bit digits: 768 bits */
typedef struct { uint32_t d[OB]; } obig;

static void ob_zero(obig* a) { memset(a, 0, sizeof(*a)); }
static void ob_add(obig* a, const obig* b) {
    uint64_t c = 0;
    for (int i = 0; i < OB; i++) {
        c += (uint64_t)a->d[i] + b->d[i];
        a->d[i] = (uint32_t)c;
        c >>= 32;
    }
}
static void ob_from_u128(obig* a, unsigned __int128 x) {
    ob_zero(a);
    for (int i = 0; i < 4; i++) { a->d[i] = (uint32_t)x; x >>= 32; }
}
static void ob_mul(const obig* a, const obig* b, obig* out) {
    obig r;
    ob_zero(&r);
    for (int i = 0; i < OB; i++) {
        uint64_t carry = 0;
        for (int j = 0; i + j < OB; j++) {
            uint64_t t = (uint64_t)a->d[i] * b->d[j] + r.d[i + j] + carry;
            r.d[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    *out = r;
}
static int ob_sub(obig* a, const obig* b) { /* a -= b; returns borrow */
    int64_t br = 0;
    for (int i = 0; i < OB; i++) {
        int64_t t = (int64_t)a->d[i] - (int64_t)b->d[i] - br;
        br = t < 0;
        a->d[i] = (uint32_t)(t + (br ? ((int64_t)1 << 32) : 0));
    }
    return (int)br;
}
static int ob_is_zero(const obig* a) {
    for (int i = 0; i < OB; i++)
        if (a->d[i]) return 0;
    return 1;
}
/* round to nearest, ties to even */
static double ob_to_double(const obig* a) {
    int top = -1;
    for (int i = OB * 32 - 1; i >= 0; i--)
        if (a->d[i / 32] >> (i % 32) & 1) { top = i; break; }
    if (top < 0) return 0.0;
    if (top < 64) {
        uint64_t v = ((uint64_t)a->d[1] << 32) | a->d[0];
        if (top < 53) return (double)v;
    }
    /* mantissa = bits top..top-52; round on bit top-53 and the sticky bits below */
    uint64_t mant = 0;
    for (int i = top; i > top - 53; i--) mant = (mant << 1) | (a->d[i / 32] >> (i % 32) & 1);
    int rb = top - 53 >= 0 ? (a->d[(top - 53) / 32] >> ((top - 53) % 32) & 1) : 0;
    int sticky = 0;
    for (int i = top - 54; i >= 0; i--)
        if (a->d[i / 32] >> (i % 32) & 1) { sticky = 1; break; }
    if (rb && (sticky || (mant & 1))) mant++;
    return ldexp((double)mant, top - 52);
}

/* ------------------------------------------------------------------ candidates */
static int has_edge(const orc_graph* g, int64_t u, int64_t x) {
    int64_t lo = g->off[u], hi = g->off[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->nbr[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < g->off[u + 1] && g->nbr[lo] == x;
}

/* S_j as an ascending list (out may be NULL); returns |S_j|. */
uint64_t orc_candidates(const orc_graph* g, const orc_plan* p, int j, const int32_t* v, int32_t* out) {
    int64_t lo = -1, hi = g->n; /* members x satisfy lo < x < hi */
    for (int i = 0; i < j; i++) {
        if (p->upper[j] >> i & 1) { if (v[i] < hi) hi = v[i]; }
        if (p->lower[j] >> i & 1) { if (v[i] > lo) lo = v[i]; }
    }
    int b = 0;
    while (!(p->connect[j] >> b & 1)) b++;
    uint64_t cnt = 0;
    for (int64_t e = g->off[v[b]]; e < g->off[v[b] + 1]; e++) {
        int32_t x = g->nbr[e];
        if (x <= lo || x >= hi) continue;
        int ok = 1;
        for (int i = 0; i < j && ok; i++) {
            if (x == v[i]) ok = 0;
            else if ((p->connect[j] >> i & 1) && !has_edge(g, v[i], x)) ok = 0;
            else if ((p->disconnect[j] >> i & 1) && has_edge(g, v[i], x)) ok = 0;
        }
        if (ok) {
            if (out) out[cnt] = x;
            cnt++;
        }
    }
    return cnt;
}

/* Measurement definition of a sample's algorithmic bytes (the work a merge
 * of sorted rows must read, independent of how a kernel does it): 8 for the
 * first edge, 16 (an int64 offset pair) for each distinct earlier vertex whose
 * row a step reads (a pattern edge or, vertex-induced, a non-edge to position
 * j), and 4 per entry of EACH such row that lies strictly inside the step's
 * symmetry-breaking bounds, for every step up to and including the first empty
 * one.  *min_b receives the same sum with only the smallest connected row's
 * entries counted (a lower bound: what a scan of the shortest row alone must
 * read). */
uint64_t orc_step_bytes(const orc_graph* g, const orc_plan* p, int j, const int32_t* v, uint32_t* opened,
                        uint64_t* min_b) {
    int64_t lo = -1, hi = g->n;
    for (int i = 0; i < j; i++) {
        if (p->upper[j] >> i & 1) { if (v[i] < hi) hi = v[i]; }
        if (p->lower[j] >> i & 1) { if (v[i] > lo) lo = v[i]; }
    }
    uint64_t b = 0, small = 0;
    uint32_t rows = (uint32_t)(p->connect[j] | p->disconnect[j]);
    for (int i = 0; i < j; i++)
        if ((rows >> i & 1) && !(*opened >> i & 1)) { b += 16; *opened |= 1u << i; }
    uint64_t head = b;
    int best = -1;
    for (int i = 0; i < j; i++) {
        if (!(rows >> i & 1)) continue;
        uint64_t in = 0;
        for (int64_t e = g->off[v[i]]; e < g->off[v[i] + 1]; e++)
            if (g->nbr[e] > lo && g->nbr[e] < hi) in += 4;
        b += in;
        if ((p->connect[j] >> i & 1) &&
            (best < 0 || g->off[v[i] + 1] - g->off[v[i]] < g->off[v[best] + 1] - g->off[v[best]])) {
            best = i;
            small = in;
        }
    }
    *min_b += head + small;
    return b;
}

void orc_ns_sample(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag, uint64_t s,
                   const uint64_t* draws, orc_rec* r) {
    memset(r, 0, sizeof(*r));
    r->s = s;
    r->k = p->k;
    for (int i = 0; i < 8; i++) r->v[i] = -1;
    uint64_t M = p->oriented ? (uint64_t)g->m : 2 * (uint64_t)g->m;
    r->size[0] = M;
    if (M == 0) { r->fail_step = 1; return; }
    uint64_t r0 = draws ? draws[0] : orc_draw(seed, s, 0, tag);
    uint64_t e = orc_mulhi(M, r0);
    if (p->oriented) { r->v[0] = g->esrc[e]; r->v[1] = g->edst[e]; }
    else { r->v[0] = g->arow[e]; r->v[1] = g->nbr[e]; }
    r->bytes = 8;
    r->bytes_min = 8;
    uint32_t opened = 0;
    unsigned __int128 alpha = M;
    int32_t* buf = NULL;
    for (int j = 2; j < p->k; j++) {
        r->bytes += orc_step_bytes(g, p, j, r->v, &opened, &r->bytes_min);
        uint64_t cnt = orc_candidates(g, p, j, r->v, NULL);
        r->size[j] = cnt;
        if (cnt == 0) {
            r->fail_step = j;
            free(buf);
            return;
        }
        buf = (int32_t*)realloc(buf, sizeof(int32_t) * (size_t)cnt);
        orc_candidates(g, p, j, r->v, buf);
        uint64_t rj = draws ? draws[j] : orc_draw(seed, s, (uint32_t)j, tag);
        r->v[j] = buf[orc_mulhi(cnt, rj)];
        unsigned __int128 next = alpha * cnt;
        if (next / cnt != alpha) r->overflow = 1;
        alpha = next;
    }
    free(buf);
    r->hit = 1;
    r->alpha_lo = (uint64_t)alpha;
    r->alpha_hi = (uint64_t)(alpha >> 64);
}

/* ------------------------------------------------------------------ NS-base
 *
 * The neighbour sampler the paper measures NS-prune against (Sec. 4.2, the
 * neighbour-sampling algorithm and its lazy verification; the comparison of
 * hit rates and convergence in the evaluation): after the same first edge,
 * position j is drawn uniformly from the UNION of the neighbourhoods of the
 * earlier positions joined to j by a pattern edge, with no other test, and
 * alpha is multiplied by the union's size; once every position is drawn, the
 * closure check tests what NS-prune tests step by step (distinct vertices, the
 * symmetry-breaking bounds, every pattern edge present and, for vertex-induced
 * counting, every non-edge absent).  A sample failing it is a miss.  Each match
 * is produced by exactly one sequence of draws, with probability 1/alpha, so
 * E[X] is the count.
 *
 * Order of the union (the index r selects into): the earlier positions joined
 * to j in ascending position, each row ascending, an entry kept at its first
 * occurrence (dropped from a later row that repeats an earlier one).
 * Status of a miss: j for an empty union at position j, k for a failed closure. */
uint64_t orc_union_candidates(const orc_graph* g, const orc_plan* p, int j, const int32_t* v, int32_t* out) {
    uint64_t cnt = 0;
    for (int i = 0; i < j; i++) {
        if (!(p->connect[j] >> i & 1)) continue;
        for (int64_t e = g->off[v[i]]; e < g->off[v[i] + 1]; e++) {
            int32_t x = g->nbr[e];
            int seen = 0;
            for (int h = 0; h < i && !seen; h++)
                if ((p->connect[j] >> h & 1) && has_edge(g, v[h], x)) seen = 1;
            if (seen) continue;
            if (out) out[cnt] = x;
            cnt++;
        }
    }
    return cnt;
}

static int closure_holds(const orc_graph* g, const orc_plan* p, const int32_t* v) {
    for (int j = 2; j < p->k; j++) {
        int64_t lo = -1, hi = g->n;
        for (int i = 0; i < j; i++) {
            if (p->upper[j] >> i & 1) { if (v[i] < hi) hi = v[i]; }
            if (p->lower[j] >> i & 1) { if (v[i] > lo) lo = v[i]; }
        }
        if (v[j] <= lo || v[j] >= hi) return 0;
        for (int i = 0; i < j; i++) {
            if (v[j] == v[i]) return 0;
            if ((p->connect[j] >> i & 1) && !has_edge(g, v[i], v[j])) return 0;
            if ((p->disconnect[j] >> i & 1) && has_edge(g, v[i], v[j])) return 0;
        }
    }
    return 1;
}

void orc_ns_base_sample(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag, uint64_t s,
                        const uint64_t* draws, orc_rec* r) {
    memset(r, 0, sizeof(*r));
    r->s = s;
    r->k = p->k;
    for (int i = 0; i < 8; i++) r->v[i] = -1;
    uint64_t M = p->oriented ? (uint64_t)g->m : 2 * (uint64_t)g->m;
    r->size[0] = M;
    if (M == 0) { r->fail_step = 1; return; }
    uint64_t r0 = draws ? draws[0] : orc_draw(seed, s, 0, tag);
    uint64_t e = orc_mulhi(M, r0);
    if (p->oriented) { r->v[0] = g->esrc[e]; r->v[1] = g->edst[e]; }
    else { r->v[0] = g->arow[e]; r->v[1] = g->nbr[e]; }
    unsigned __int128 alpha = M;
    int32_t* buf = NULL;
    for (int j = 2; j < p->k; j++) {
        uint64_t cnt = orc_union_candidates(g, p, j, r->v, NULL);
        r->size[j] = cnt;
        if (cnt == 0) {
            r->fail_step = j;
            free(buf);
            return;
        }
        buf = (int32_t*)realloc(buf, sizeof(int32_t) * (size_t)cnt);
        orc_union_candidates(g, p, j, r->v, buf);
        uint64_t rj = draws ? draws[j] : orc_draw(seed, s, (uint32_t)j, tag);
        r->v[j] = buf[orc_mulhi(cnt, rj)];
        unsigned __int128 next = alpha * cnt;
        if (next / cnt != alpha) r->overflow = 1;
        alpha = next;
    }
    free(buf);
    if (!closure_holds(g, p, r->v)) {
        r->fail_step = p->k;
        return;
    }
    r->hit = 1;
    r->alpha_lo = (uint64_t)alpha;
    r->alpha_hi = (uint64_t)(alpha >> 64);
}

/* SplitMix64 finaliser (Steele, Lea, Flood 2014). */
static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Record hash; the run checksum is the sum of these mod 2^64. */
uint64_t orc_rec_hash(const orc_rec* r) {
    uint64_t h = mix64(r->s ^ 0x9E3779B97F4A7C15ULL);
    uint64_t status = r->hit ? 0xFFu : (uint64_t)r->fail_step;
    h = mix64(h ^ status);
    int filled = r->hit ? r->k : r->fail_step;
    for (int i = 0; i < r->k; i++) {
        uint32_t vi = i < filled ? (uint32_t)r->v[i] : 0xFFFFFFFFu;
        h = mix64(h ^ (uint64_t)vi);
    }
    h = mix64(h ^ r->alpha_lo);
    h = mix64(h ^ r->alpha_hi);
    return h;
}

typedef struct {
    const orc_graph* g; const orc_plan* p; uint64_t seed; uint32_t tag;
    uint64_t s0, s1; orc_rec* out; int base; /* 1: NS-base, else NS-prune */
    obig S1, S2; uint64_t hits, checksum, bytes; int overflow;
} ns_job;

static void* ns_worker(void* arg) {
    ns_job* J = (ns_job*)arg;
    ob_zero(&J->S1); ob_zero(&J->S2);
    J->hits = 0; J->checksum = 0; J->bytes = 0; J->overflow = 0;
    orc_rec r;
    for (uint64_t s = J->s0; s < J->s1; s++) {
        if (J->base) orc_ns_base_sample(J->g, J->p, J->seed, J->tag, s, NULL, &r);
        else orc_ns_sample(J->g, J->p, J->seed, J->tag, s, NULL, &r);
        if (J->out) J->out[s - J->s0] = r;
        J->checksum += orc_rec_hash(&r);
        J->bytes += r.bytes;
        J->overflow |= r.overflow;
        if (r.hit) {
            J->hits++;
            unsigned __int128 a = ((unsigned __int128)r.alpha_hi << 64) | r.alpha_lo;
            obig x, x2;
            ob_from_u128(&x, a);
            ob_mul(&x, &x, &x2);
            ob_add(&J->S1, &x);
            ob_add(&J->S2, &x2);
        }
    }
    return NULL;
}

static void run_range(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag, uint64_t s0,
                      uint64_t count, int nthreads, orc_rec* out, ns_job* total, int base) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    ns_job jobs[64];
    for (int t = 0; t < nthreads; t++) {
        jobs[t].g = g; jobs[t].p = p; jobs[t].seed = seed; jobs[t].tag = tag;
        jobs[t].s0 = s0 + count * (uint64_t)t / (uint64_t)nthreads;
        jobs[t].s1 = s0 + count * (uint64_t)(t + 1) / (uint64_t)nthreads;
        jobs[t].out = out ? out + (jobs[t].s0 - s0) : NULL;
        jobs[t].base = base;
        pthread_create(&th[t], NULL, ns_worker, &jobs[t]);
    }
    ob_zero(&total->S1); ob_zero(&total->S2);
    total->hits = 0; total->checksum = 0; total->bytes = 0; total->overflow = 0;
    for (int t = 0; t < nthreads; t++) {
        pthread_join(th[t], NULL);
        ob_add(&total->S1, &jobs[t].S1);
        ob_add(&total->S2, &jobs[t].S2);
        total->hits += jobs[t].hits;
        total->checksum += jobs[t].checksum;
        total->bytes += jobs[t].bytes;
        total->overflow |= jobs[t].overflow;
    }
}

int orc_ns_trace(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag, uint64_t s0,
                 uint64_t count, int nthreads, orc_rec* out) {
    ns_job total;
    run_range(g, p, seed, tag, s0, count, nthreads, out, &total, 0);
    return 0;
}

int orc_ns_base_trace(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag, uint64_t s0,
                      uint64_t count, int nthreads, orc_rec* out) {
    ns_job total;
    run_range(g, p, seed, tag, s0, count, nthreads, out, &total, 1);
    return 0;
}

/* ------------------------------------------------------------------ statistics */

/* Phi^-1(p) for 0.5 < p < 1 by bisection on Phi(x) = erfc(-x/sqrt 2)/2,
 * evaluated in x87 extended precision so the result is within an ulp. */
double orc_norm_ppf(double p) {
    if (!(p > 0.5 && p < 1.0)) return NAN;
    long double lo = 0.0L, hi = 40.0L, P = (long double)p;
    for (int it = 0; it < 4000; it++) {
        long double mid = 0.5L * (lo + hi);
        if (mid == lo || mid == hi) break;
        long double f = 0.5L * erfcl(-mid / sqrtl(2.0L));
        if (f < P) lo = mid; else hi = mid;
    }
    return (double)(0.5L * (lo + hi));
}

/* Correctly rounded double of a little-endian 32-bit digit integer. */
double orc_digits_to_double(const uint32_t* d, int nd) {
    obig a;
    ob_zero(&a);
    for (int i = 0; i < nd && i < OB; i++) a.d[i] = d[i];
    return ob_to_double(&a);
}

double orc_eps_hat(double z, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2) {
    obig S1, S2, N, a, b;
    ob_zero(&S1); ob_zero(&S2); ob_zero(&N);
    for (int i = 0; i < n1 && i < OB; i++) S1.d[i] = s1[i];
    for (int i = 0; i < n2 && i < OB; i++) S2.d[i] = s2[i];
    if (ob_is_zero(&S1) || n == 0) return INFINITY;
    N.d[0] = (uint32_t)n; N.d[1] = (uint32_t)(n >> 32);
    ob_mul(&N, &S2, &a);   /* n * S2 */
    ob_mul(&S1, &S1, &b);  /* S1^2 */
    if (ob_sub(&a, &b)) return NAN; /* impossible by Cauchy-Schwarz */
    double D = ob_to_double(&a), dn = (double)n, dS1 = ob_to_double(&S1);
    double q = D / dn;
    double r = sqrt(q);
    double t = z * r;
    return t / dS1;
}

/* Student's t distribution with nu degrees of freedom: P(|T| <= t) by the
 * closed forms for integer nu (Abramowitz and Stegun 26.7.3 for odd nu,
 * 26.7.4 for even nu), with theta = atan(t / sqrt(nu)):
 *   odd nu:  (2/pi) [theta + sin(theta) (cos + (2/3) cos^3 + (2*4)/(3*5) cos^5
 *            + ... up to cos^(nu-2))]   (theta alone for nu = 1)
 *   even nu: sin(theta) [1 + (1/2) cos^2 + (1*3)/(2*4) cos^4 + ... up to cos^(nu-2)]
 * evaluated in x87 extended precision. */
static long double t_central(long double t, int nu) {
    long double th = atanl(t / sqrtl((long double)nu)), s = sinl(th), c = cosl(th);
    if (nu % 2) {
        long double sum = 0.0L;
        if (nu > 1) {
            long double term = c;   /* cos^1 */
            sum = term;
            for (int i = 3; i <= nu - 2; i += 2) {
                term *= c * c * (long double)(i - 1) / (long double)i;
                sum += term;
            }
        }
        return 2.0L / 3.14159265358979323846264338327950288L * (th + s * sum);
    }
    long double term = 1.0L, sum = 1.0L;
    for (int i = 2; i <= nu - 2; i += 2) {
        term *= c * c * (long double)(i - 1) / (long double)i;
        sum += term;
    }
    return s * sum;
}

/* t with P(|T| <= t) = conf for nu degrees of freedom (the two-sided quantile,
 * t_{nu}(1 - delta/2) with conf = 1 - delta), by bisection in extended
 * precision, then rounded to double. */
double orc_t_ppf(double conf, int nu) {
    if (!(conf > 0.0 && conf < 1.0) || nu < 1) return NAN;
    long double lo = 0.0L, hi = 1.0L, C = (long double)conf;
    while (t_central(hi, nu) < C) hi *= 2.0L;
    for (int it = 0; it < 20000; it++) {
        long double mid = 0.5L * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (t_central(mid, nu) < C) lo = mid; else hi = mid;
    }
    return (double)(0.5L * (lo + hi));
}

/* Predicted relative error of the mean of n i.i.d. values from their exact
 * sums with the unbiased sample variance s^2 = (S2 - S1^2/n) / (n - 1): the
 * standard error over the mean is sqrt(D / (n - 1)) / S1 with D = n S2 - S1^2,
 * scaled by the t quantile.  +inf while n < 2 or S1 = 0.  Used for the repeated
 * sparsifications of the GS path, where n is small. */
double orc_eps_hat_t(double t, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2) {
    obig S1, S2, N, a, b;
    ob_zero(&S1); ob_zero(&S2); ob_zero(&N);
    for (int i = 0; i < n1 && i < OB; i++) S1.d[i] = s1[i];
    for (int i = 0; i < n2 && i < OB; i++) S2.d[i] = s2[i];
    if (ob_is_zero(&S1) || n < 2) return INFINITY;
    N.d[0] = (uint32_t)n; N.d[1] = (uint32_t)(n >> 32);
    ob_mul(&N, &S2, &a);
    ob_mul(&S1, &S1, &b);
    if (ob_sub(&a, &b)) return NAN;
    double D = ob_to_double(&a), dn1 = (double)(n - 1), dS1 = ob_to_double(&S1);
    double q = D / dn1;
    double r = sqrt(q);
    double u = t * r;
    return u / dS1;
}

static uint64_t round_up(uint64_t x, uint64_t q) { return q ? (x + q - 1) / q * q : x; }

/* Window schedule: n_0 = n_min; n_{t+1} = n_t + max(w_min, ceil(growth * n_t)),
 * each rounded up to the quantum and clamped to max_samples. */
uint64_t orc_window_next(uint64_t n_t, const orc_ns_opts* o) {
    uint64_t nx;
    if (n_t == 0) nx = round_up(o->n_min, o->quantum);
    else {
        double gr = ceil(o->growth * (double)n_t);
        uint64_t inc = (uint64_t)gr;
        if (inc < o->w_min) inc = o->w_min;
        nx = round_up(n_t + inc, o->quantum);
    }
    if (o->max_samples && nx > o->max_samples) nx = o->max_samples;
    return nx;
}

static void store_digits(const obig* a, uint32_t* out, int nd, int* overflow) {
    for (int i = 0; i < nd; i++) out[i] = a->d[i];
    for (int i = nd; i < OB; i++)
        if (a->d[i]) *overflow = 1;
}

int orc_ns_run(const orc_graph* g, const orc_plan* p, const orc_ns_opts* o, orc_ns_result* res,
               double* eps_trace, uint64_t* n_trace, int trace_cap) {
    memset(res, 0, sizeof(*res));
    double z = orc_norm_ppf(1.0 - (1.0 - o->confidence) / 2.0);
    res->z = z;
    uint64_t M = p->oriented ? (uint64_t)g->m : 2 * (uint64_t)g->m;
    if (M == 0) { res->converged = 1; res->estimate = 0.0; res->eps_hat = 0.0; return 0; }
    obig S1, S2;
    ob_zero(&S1); ob_zero(&S2);
    uint64_t n = 0;
    int t = 0;
    for (;;) {
        uint64_t nx = o->fixed_n ? o->fixed_n : orc_window_next(n, o);
        if (nx <= n) break;
        ns_job part;
        run_range(g, p, o->seed, o->tag, n, nx - n, o->nthreads, NULL, &part, o->sampler == 1);
        ob_add(&S1, &part.S1);
        ob_add(&S2, &part.S2);
        res->hits += part.hits;
        res->checksum += part.checksum;
        res->bytes += part.bytes;
        res->overflow |= part.overflow;
        n = nx;
        t++;
        double eh = orc_eps_hat(z, n, S1.d, OB, S2.d, OB);
        if (eps_trace && t <= trace_cap) { eps_trace[t - 1] = eh; n_trace[t - 1] = n; }
        res->eps_hat = eh;
        if (o->fixed_n) break;
        if (eh <= o->eps) { res->converged = 1; break; }
        if (o->max_samples && n >= o->max_samples) break;
    }
    res->n = n;
    res->windows = t;
    res->estimate = ob_to_double(&S1) / (double)n;
    store_digits(&S1, res->s1, 8, &res->overflow);
    store_digits(&S2, res->s2, 12, &res->overflow);
    if (o->fixed_n && res->eps_hat <= o->eps) res->converged = 1;
    return 0;
}
