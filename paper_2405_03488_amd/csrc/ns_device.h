// Device-side NS-prune sampler shared by the window kernels and the persistent
// batch kernel.  See ns_kernels.hip for the sampling definition.
#pragma once
#include "sgpm_internal.h"

namespace sgpm {

__device__ __forceinline__ uint64_t philox_r64(uint64_t seed, uint64_t s, uint32_t d, uint32_t tag) {
    uint32_t c0 = (uint32_t)s, c1 = (uint32_t)(s >> 32), c2 = d, c3 = tag;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return ((uint64_t)c1 << 32) | (uint64_t)c0;
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014), used by the record hash.
__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// first index in [lo, hi) of the ascending row with row[i] >= x
__device__ __forceinline__ int32_t lower_bound(const int32_t* __restrict__ row, int32_t lo, int32_t hi, int32_t x) {
    while (lo < hi) {
        const int32_t mid = (int32_t)(((uint32_t)lo + (uint32_t)hi) >> 1);
        if (row[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void add_carry(uint64_t& acc, uint64_t x, uint64_t& carry) {
    const uint64_t t = acc + x;
    const uint64_t c1 = t < x;
    const uint64_t t2 = t + carry;
    const uint64_t c2 = t2 < carry;
    acc = t2;
    carry = c1 + c2;
}

struct Acc {
    uint64_t s1[3];   // sum X, 192 bits
    uint64_t s2[5];   // sum X^2, 320 bits
    uint64_t hits, csum, bytes, ovf;
};

__device__ __forceinline__ void acc_add(Acc& a, uint64_t lo, uint64_t hi) {
    uint64_t c = 0;
    add_carry(a.s1[0], lo, c);
    add_carry(a.s1[1], hi, c);
    a.s1[2] += c;
    // X^2 = lo^2 + 2 lo hi 2^64 + hi^2 2^128
    uint64_t w0 = lo * lo, w1 = __umul64hi(lo, lo), w2 = 0, w3 = 0;
    if (hi) {
        const uint64_t m0 = lo * hi, m1 = __umul64hi(lo, hi);
        const uint64_t d0 = m0 << 1, d1 = (m1 << 1) | (m0 >> 63), d2 = m1 >> 63;
        const uint64_t h0 = hi * hi, h1 = __umul64hi(hi, hi);
        uint64_t cc = 0;
        add_carry(w1, d0, cc);
        w2 = d1;
        add_carry(w2, h0, cc);
        w3 = d2;
        add_carry(w3, h1, cc);
    }
    c = 0;
    add_carry(a.s2[0], w0, c);
    add_carry(a.s2[1], w1, c);
    add_carry(a.s2[2], w2, c);
    add_carry(a.s2[3], w3, c);
    a.s2[4] += c;
}

constexpr int32_t BIG = 0x7FFFFFFF;

// With one sample per wave (G = 64) every per-sample value is wave-uniform;
// readfirstlane tells the compiler so, which keeps the walk state in SGPRs
// and turns its branches into scalar branches.
__device__ __forceinline__ int32_t rfl(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t rfl64(int64_t x) {
    return (int64_t)(((uint64_t)(uint32_t)rfl((int32_t)((uint64_t)x >> 32)) << 32) | (uint32_t)rfl((int32_t)x));
}
template <int G>
__device__ __forceinline__ int32_t uni(int32_t x) {
    if constexpr (G == 64) return rfl(x);
    else return x;
}
// The value of v in lane `src` (an absolute lane of the wave).  One sample per
// wave (G = 64): src is wave-uniform and the value comes back by readlane,
// with no LDS round trip; a group of G < 64 lanes uses a lane permute.
template <int G>
__device__ __forceinline__ int32_t from_lane(int32_t v, int src) {
    if constexpr (G == 64) return __builtin_amdgcn_readlane(v, src);
    else return __shfl(v, src);
}

// candidate lists per block (14 KB): with the records and sums, eight
// one-sample-per-wave blocks fit a CU's 160 KB of LDS
constexpr int LDS_WORDS = 3584;

// first index in [lo, hi) with row[i] >= x, galloping forward from lo
__device__ __forceinline__ int32_t gallop(const int32_t* __restrict__ row, int32_t lo, int32_t hi, int32_t x) {
    if (lo >= hi || row[lo] >= x) return lo;
    int32_t prev = lo, step = 1;
    for (;;) {
        const int32_t nxt = prev + step;
        if (nxt >= hi) return lower_bound(row, prev + 1, hi, x);
        if (row[nxt] >= x) return lower_bound(row, prev + 1, nxt, x);
        prev = nxt;
        step <<= 1;
    }
}

template <int G>
__device__ __forceinline__ uint64_t group_ballot(bool pred, uint64_t gmask) {
    return __ballot(pred) & gmask;
}

// Membership of each lane's x in the ascending row R[0, rl) for a group whose
// active lanes hold ascending values (xmax = the largest).  The group-uniform
// cursor c only moves forward: entries before it are below every x still to
// come.  G = 1: galloping search.  G > 1: the group loads G consecutive row
// entries, every lane binary-searches its x among them through shuffles, and
// the window slides until no active lane's x lies beyond it; across a long gap
// (a hub's row against a few candidates) it jumps by a G-ary search.
template <int G>
__device__ __forceinline__ bool member(const int32_t* __restrict__ R, int32_t rl, int32_t& c, int32_t x, bool act,
                                       int32_t xmax, int gbase, int gl, uint64_t gmask) {
    if constexpr (G == 1) {
        if (!act) return false;
        const int32_t q = gallop(R, c, rl, x);
        c = q;
        return q < rl && R[q] == x;
    } else {
        bool found = false, pending = act;
        int32_t b = (c + gl < rl) ? R[c + gl] : BIG;
        for (;;) {
            const int32_t bmax = uni<G>(from_lane<G>(b, gbase + G - 1));
            // binary search of x in the window through lane permutes, the
            // position kept as the permute's byte address (lane * 4); a
            // position of G (every entry below x) reads another lane, and the
            // test below ignores it
            int pb = gbase * 4;
#pragma unroll
            for (int st = G / 2; st >= 1; st >>= 1) {
                const int32_t bv = __builtin_amdgcn_ds_bpermute(pb + (st - 1) * 4, b);
                pb += bv < x ? st * 4 : 0;
            }
            const int pos = (pb >> 2) - gbase;
            const int32_t bq = __builtin_amdgcn_ds_bpermute(pb, b);
            const bool res = pending && x <= bmax;
            if (res) found = pos < G && bq == x;
            pending = pending && !res;
            const uint64_t pend = group_ballot<G>(pending, gmask);
            if (pend == 0) {
                c += (int32_t)__popcll(group_ballot<G>(b < xmax, gmask));
                break;
            }
            const bool below = group_ballot<G>(res, gmask) == 0;  // the window lies below every pending x
            c += G;
            const int32_t xmin = below && rl - c > 8 * G ? uni<G>(from_lane<G>(x, __ffsll((unsigned long long)pend) - 1)) : 0;
            if (below && rl - c > 8 * G && uni<G>(R[c + 8 * G - 1]) < xmin) {
                // more than 8 windows from the smallest pending x: a G-ary search
                // for the first entry >= it, each round probing G evenly spaced
                // entries and keeping the gap that holds it, so a long row costs
                // a few round trips, not one per G entries.  Entries skipped are
                // below every x still pending.  (A single probe 8 windows ahead
                // keeps short gaps on the cheaper slide.)
                int32_t lo = c + 8 * G, hi = rl;  // the entry sought lies in [lo, hi]
                while (hi - lo > G) {
                    const int32_t step = (hi - lo) / G;
                    const int32_t pv = R[lo + (gl + 1) * step - 1];
                    const int nb = (int)__popcll(group_ballot<G>(pv < xmin, gmask));
                    if (nb < G) hi = lo + (nb + 1) * step - 1;
                    lo += nb * step;
                }
                c = lo;
            }
            b = (c + gl < rl) ? R[c + gl] : BIG;
        }
        return found;
    }
}

// One NS-prune sample.  Returns 0xFF for a hit, else the failing position j.
// For G > 1 all G lanes of a group call it with the same s.  `list` is the
// group's LDS area of CAP words holding the current candidate set.
// Degree bucket floor(log2(1 + d)), clipped to 31: of an embedded vertex from
// its row length (already loaded), of a candidate from the graph's byte array.
__device__ __forceinline__ int32_t bucket_of_degree(int32_t d) {
    const int32_t b = 31 - (int32_t)__clz((uint32_t)d + 1u);
    return b < 31 ? b : 31;
}
__device__ __forceinline__ int32_t bucket_of(const LearnArgs& la, int32_t x) { return (int32_t)la.vb[x]; }

// Inclusive prefix sums over lanes 0-31 (two rows of 16 lanes): DPP shifts by
// 1, 2, 4 and 8 within each row, then row 0's total broadcast into row 1.
// Lanes 32-63 end with sums of their own rows (callers ignore them).  Every
// lane of the wave must be active.
__device__ __forceinline__ uint32_t scan32_dpp(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, (unsigned)o);
        if (lane >= o) x += y;
    }
    return x;
}

// alpha' * 2^52 as an exact 128-bit integer (alpha' >= 1); false when alpha' >= 2^76
__device__ __forceinline__ bool fixed52(double a, uint64_t& lo, uint64_t& hi) {
    if (!(a < 75557863725914323419136.0)) return false;  // 2^76
    const uint64_t bits = (uint64_t)__double_as_longlong(a);
    const int e = (int)((bits >> 52) & 0x7FF) - 1023;
    const uint64_t mant = (bits & ((1ull << 52) - 1ull)) | (1ull << 52);
    if (e < 64) {
        lo = mant << e;
        hi = e == 0 ? 0ull : mant >> (64 - e);
    } else {
        lo = 0;
        hi = mant << (e - 64);
    }
    return true;
}

// Draws computed ahead, one per lane (the wave kernel evaluates all draws of a
// group of samples at once).  Slot t of the current sample sits in lane
// base + t: slots 0..k-2 hold draws 0, 2, .., k-1, slots k-1.. draws 18, 19, ..
// A sample's first edge and the bounds of its two rows, loaded ahead by the
// group prologue (one lane per sample, so the group's loads overlap).
struct Head {
    int32_t v0, v1;
    int64_t b0, b1;
    int32_t l0, l1;
    int32_t k0, k1;  // learned proposal: degree buckets of v0 and v1
};

struct Draws {
    uint32_t lo, hi;  // this lane's draw
    int base;         // lane of slot 0 of the current sample
    int k1;           // k - 1
};

// Draw d of sample s: read from the lanes holding it, or computed here.
__device__ __forceinline__ uint64_t draw_at(const Draws* dr, uint64_t seed, uint64_t s, uint32_t d, uint32_t tag) {
    if (!dr) return philox_r64(seed, s, d, tag);
    const int slot = d == 0 ? 0 : d < 16 ? (int)d - 1 : dr->k1 + (int)d - 18;
    const int l = dr->base + slot;
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)dr->hi, l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)dr->lo, l);
}

// CLQ: the plan is known to be the k-clique's (connect[j] = upper[j] = all
// earlier positions, no disconnect or lower bounds, oriented first edge, S_j
// filtered from S_{j-1} from j = 3 on), so every plan test folds at compile
// time; the caller checks the plan before choosing it.
template <int G, int KMAX = 8, bool CLQ = false>
__device__ __forceinline__ uint32_t ns_sample(const DGraph& g, const Plan& p, uint64_t seed, uint32_t tag, uint64_t s,
                                             int32_t (&v)[8], uint64_t& alo, uint64_t& ahi, uint64_t& ovf,
                                             uint64_t& bytes, bool count_bytes, int32_t* list,
                                             const LearnArgs* la = nullptr, uint32_t* hist = nullptr,
                                             uint32_t* sz = nullptr, const Draws* dr = nullptr,
                                             const Head* hd = nullptr) {
    constexpr int CAP = LDS_WORDS / (256 / G);
    const int lane = (int)(threadIdx.x & 63);
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
    const uint64_t below = (1ull << lane) - 1ull;

#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = -1;
    const bool oriented = CLQ || p.oriented;
    const int pk = CLQ ? KMAX : p.k;
    const uint64_t M = oriented ? (uint64_t)g.m : 2ull * (uint64_t)g.m;
    const int32_t* rp[8];
    int32_t rl[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        rp[i] = nullptr;
        rl[i] = 0;
    }
    if (hd) {
        v[0] = hd->v0;
        v[1] = hd->v1;
        rp[0] = g.nbr + hd->b0;
        rl[0] = hd->l0;
        rp[1] = g.nbr + hd->b1;
        rl[1] = hd->l1;
    } else {
        const uint64_t e = __umul64hi(M, draw_at(dr, seed, s, 0, tag));
        if (oriented) {
            const int2 pr = g.epair[e];
            v[0] = pr.x;
            v[1] = pr.y;
        } else {
            v[0] = g.arow[e];
            v[1] = g.nbr[e];
        }
        const int64_t b0 = g.off[v[0]], e0 = g.off[v[0] + 1];
        const int64_t b1 = g.off[v[1]], e1 = g.off[v[1] + 1];
        rp[0] = g.nbr + b0;
        rl[0] = (int32_t)(e0 - b0);
        rp[1] = g.nbr + b1;
        rl[1] = (int32_t)(e1 - b1);
    }
    alo = M;
    ahi = 0;
    bytes = 8;
    const bool learned = (G == 64) && la != nullptr && la->table != nullptr;
    double af = (double)M;
    int32_t b0 = 0;
    if (learned) b0 = hd ? hd->k0 : bucket_of_degree(rl[0]);
    uint32_t opened = 0;
    int32_t prevcnt = -1;  // |S_{j-1}| when the whole set sits in `list`

#pragma unroll
    for (int j = 2; j < KMAX; ++j) {
        if (j >= pk) break;
        const uint32_t conn = CLQ ? (1u << j) - 1u : (uint32_t)p.connect[j];
        const uint32_t disc = CLQ ? 0u : (uint32_t)p.disconnect[j];
        const uint32_t up = CLQ ? (1u << j) - 1u : (uint32_t)p.upper[j];
        const uint32_t lw = CLQ ? 0u : (uint32_t)p.lower[j];
        int32_t lo = -1, hi = BIG;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            if (up >> i & 1) hi = min(hi, v[i]);
            if (lw >> i & 1) lo = max(lo, v[i]);
        }
        // learned proposal: this step's weight-table row, loaded while the
        // candidates are scanned
        // (the last step picks uniformly: every candidate completes exactly one match)
        const bool weighted = learned && j + 1 < pk;
        uint32_t wrow = 0;
        if (weighted && lane < 32) {
            const int32_t bp = (j == 2 && hd) ? hd->k1 : bucket_of_degree(rl[j - 1]);
            wrow = (uint32_t)la->table[(((size_t)j * 32 + (size_t)b0) * 32 + (size_t)bp) * 32 + lane];
        }
        // smallest connected earlier row (lowest position on ties)
        int d = -1;
        int32_t dl = BIG;
        const int32_t* dp = nullptr;
#pragma unroll
        for (int i = 0; i < j; ++i)
            if ((conn >> i & 1) && rl[i] < dl) {
                d = i;
                dl = rl[i];
                dp = rp[i];
            }
        if (count_bytes) {
            // 16 per newly opened row, 4 per entry inside (lo, hi) of every row
            // the step merges (connected and, vertex-induced, disconnected)
            const uint32_t rows = conn | disc;
#pragma unroll
            for (int i = 0; i < j; ++i)
                if (rows >> i & 1) {
                    if (!(opened >> i & 1)) {
                        bytes += 16;
                        opened |= 1u << i;
                    }
                    const int32_t w0 = lo >= 0 ? lower_bound(rp[i], 0, rl[i], lo + 1) : 0;
                    const int32_t w1 = hi < BIG ? lower_bound(rp[i], w0, rl[i], hi) : rl[i];
                    bytes += 4ull * (uint64_t)(w1 - w0);
                }
        }
        // Reuse: when step j's constraints contain step j-1's, S_j is the part
        // of S_{j-1} (already in `list`) that meets the extra constraints.
        const bool reuse = (j >= 3) && (CLQ || p.reuse[j]) && prevcnt >= 0;
        uint32_t need_conn, need_disc, excl;
        const int32_t* src;
        int32_t slen, start;
        if (reuse) {
            need_conn = conn & ~(CLQ ? (1u << (j - 1)) - 1u : (uint32_t)p.connect[j - 1]);
            need_disc = CLQ ? 0u : disc & ~(uint32_t)p.disconnect[j - 1];
            excl = (1u << (j - 1)) & ~conn;
            src = list;
            slen = prevcnt;
            start = 0;
        } else {
            need_conn = conn & ~(1u << d);
            need_disc = disc;
            excl = ((1u << j) - 1u) & ~conn;
            src = dp;
            slen = dl;
            start = lo >= 0 ? lower_bound(dp, 0, dl, lo + 1) : 0;
        }
        int32_t cur[8];
        // candidates of one chunk of G source entries; advances the cursors
        auto eval_chunk = [&](int32_t base, int32_t& x, uint64_t& inm) -> bool {
            const uint32_t need = need_conn | need_disc;
            const int32_t pos = base + gl;
            x = pos < slen ? src[pos] : BIG;
            const bool act = x < hi;
            inm = group_ballot<G>(act, gmask);
            bool ok = act && x > lo;
#pragma unroll
            for (int i = 0; i < j; ++i)
                if (excl >> i & 1) ok = ok && (x != v[i]);
            if (inm == 0) return false;
            const int32_t xmax = uni<G>(from_lane<G>(x, gbase + (int)__popcll(inm) - 1));
#pragma unroll
            for (int i = 0; i < j; ++i) {
                if (need >> i & 1) {
                    const bool f = member<G>(rp[i], rl[i], cur[i], x, act, xmax, gbase, gl, gmask);
                    ok = ok && ((need_conn >> i & 1) ? f : !f);
                }
            }
            return ok;
        };

        // count pass; candidates are appended to `list` while they fit (in place
        // when reusing: a chunk is read before any of its slots is rewritten)
#pragma unroll
        for (int i = 0; i < 8; ++i) cur[i] = 0;
        uint32_t cnt = 0;
        for (int32_t base = start; base < slen; base += G) {
            int32_t x;
            uint64_t inm;
            const bool ok = eval_chunk(base, x, inm);
            const uint64_t okm = group_ballot<G>(ok, gmask);
            const uint32_t rank = (uint32_t)__popcll(okm & below);
            if (ok && cnt + rank < (uint32_t)CAP) list[cnt + rank] = x;
            cnt += (uint32_t)__popcll(okm);
            if (inm != gmask) break;
        }
        if (sz) sz[j] = cnt;
        if (cnt == 0) return (uint32_t)j;

        uint32_t idx = 0;
        if constexpr (G == 64) {
            if (learned && !weighted) {
                idx = (uint32_t)__umul64hi((uint64_t)cnt, draw_at(dr, seed, s, (uint32_t)j, tag));
                af = __dmul_rn(af, (double)cnt);
            } else if (weighted && cnt <= (uint32_t)CAP) {
                // Bucket counts from the list's order: buckets do not increase
                // with the id, so in the ascending list each bucket is one run.
                // Lane b < 32 finds the first candidate of bucket <= b by a
                // binary search for the first id of those buckets (lane_thr),
                // and n_b is its distance to lane b-1's position.
                int32_t lo = 0;
                if (lane < 32) {
                    int32_t hi = (int32_t)cnt;
                    const int32_t thr = la->lane_thr;
                    while (lo < hi) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (list[mid] < thr) lo = mid + 1;
                        else hi = mid;
                    }
                }
                const int32_t before = __shfl(lo, lane - 1);
                const uint32_t nb = lane < 32 ? (uint32_t)((lane == 0 ? (int32_t)cnt : before) - lo) : 0u;
                if (__popcll(__ballot(nb != 0u)) == 1) {
                    // every candidate in one bucket: the weighted choice reduces to
                    // a uniform member drawn with draw 16+j, and the factor
                    // sum / w_b is exactly |S_j|
                    idx = (uint32_t)__umul64hi((uint64_t)cnt, draw_at(dr, seed, s, 16u + (uint32_t)j, tag));
                    af = __dmul_rn(af, (double)cnt);
                } else {
                    // weighted bucket, then a uniform member of it: counts n_b <= CAP
                    // and n_b w_b < 2^26, so both running sums fit 32 bits; bucket b
                    // sits in lane b and the sums are scanned with DPP row shifts
                    const uint32_t w = (uint32_t)wrow;
                    const uint32_t cum = scan32_dpp(nb * w), cumn = scan32_dpp(nb);
                    const uint64_t sigma = (uint32_t)__builtin_amdgcn_readlane((int)cum, 31);
                    const uint64_t t = __umul64hi(sigma, draw_at(dr, seed, s, (uint32_t)j, tag));
                    const int bsel = __ffsll((unsigned long long)__ballot(lane < 32 && (uint64_t)cum > t)) - 1;
                    const uint64_t nbs = (uint32_t)__builtin_amdgcn_readlane((int)nb, bsel);
                    const uint64_t wbs = (uint32_t)__builtin_amdgcn_readlane((int)w, bsel);
                    const uint64_t upto = (uint32_t)__builtin_amdgcn_readlane((int)cumn, bsel);
                    const uint64_t inb = __umul64hi(nbs, draw_at(dr, seed, s, 16u + (uint32_t)j, tag));
                    idx = (uint32_t)((uint64_t)cnt - upto + inb);
                    af = __dmul_rn(af, __ddiv_rn((double)sigma, (double)wbs));
                }
            } else if (weighted) {
                // the same when the set overflowed the list: histogram by rescanning
                if (lane < 32) hist[lane] = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) cur[i] = 0;
                for (int32_t base = start; base < slen; base += G) {
                    int32_t x;
                    uint64_t inm;
                    const bool ok = eval_chunk(base, x, inm);
                    if (ok) atomicAdd(&hist[bucket_of(*la, x)], 1u);
                    if (inm != gmask) break;
                }
                const uint64_t nb = lane < 32 ? (uint64_t)hist[lane] : 0ull;
                const uint64_t w = (uint64_t)wrow;
                const uint64_t cum = wave_incl_scan(nb * w);
                const uint64_t cumn = wave_incl_scan(nb);
                const uint64_t sigma = __shfl(cum, 63);
                const uint64_t t = __umul64hi(sigma, draw_at(dr, seed, s, (uint32_t)j, tag));
                const int bsel = __ffsll((unsigned long long)__ballot(lane < 32 && cum > t)) - 1;
                const uint64_t nbs = __shfl(nb, bsel), wbs = __shfl(w, bsel), upto = __shfl(cumn, bsel);
                const uint64_t inb = __umul64hi(nbs, draw_at(dr, seed, s, 16u + (uint32_t)j, tag));
                idx = (uint32_t)((uint64_t)cnt - upto + inb);
                af = __dmul_rn(af, __ddiv_rn((double)sigma, (double)wbs));
            } else {
                idx = (uint32_t)__umul64hi((uint64_t)cnt, draw_at(dr, seed, s, (uint32_t)j, tag));
            }
        } else {
            idx = (uint32_t)__umul64hi((uint64_t)cnt, draw_at(dr, seed, s, (uint32_t)j, tag));
        }
        int32_t pick = -1;
        if (cnt <= (uint32_t)CAP) {
            pick = uni<G>(list[idx]);
            prevcnt = (int32_t)cnt;
        } else {
            // the set overflowed the list (never when reusing): select by rescanning
#pragma unroll
            for (int i = 0; i < 8; ++i) cur[i] = 0;
            uint32_t seen = 0;
            for (int32_t base = start; base < slen; base += G) {
                int32_t x;
                uint64_t inm;
                const bool ok = eval_chunk(base, x, inm);
                uint64_t okm = group_ballot<G>(ok, gmask);
                const uint32_t c = (uint32_t)__popcll(okm);
                if (seen + c > idx) {
                    for (uint32_t t = idx - seen; t > 0; --t) okm &= okm - 1ull;
                    pick = uni<G>(from_lane<G>(x, __ffsll((unsigned long long)okm) - 1));
                    break;
                }
                seen += c;
                if (inm != gmask) break;
            }
            prevcnt = -1;
        }
        if (pick < 0) {  // count and select passes disagree: report, never index with it
            ovf = 1;
            return (uint32_t)j;
        }
        v[j] = pick;
        if (j + 1 < pk) {
            const int64_t bj = g.off[pick], ej = g.off[pick + 1];
            rp[j] = g.nbr + bj;
            rl[j] = (int32_t)(ej - bj);
        }
        if (!learned) {
            // alpha *= |S_j| with 128-bit overflow detection
            const uint64_t plo = alo * (uint64_t)cnt, phi = __umul64hi(alo, (uint64_t)cnt);
            const uint64_t qlo = ahi * (uint64_t)cnt, qhi = __umul64hi(ahi, (uint64_t)cnt);
            const uint64_t nhi = phi + qlo;
            if (qhi != 0 || nhi < qlo) ovf = 1;
            alo = plo;
            ahi = nhi;
        }
    }
    if (learned) {
        if (!fixed52(af, alo, ahi)) {
            ovf = 1;
            alo = ahi = 0;
        }
    }
    return 0xFFu;
}

// Group prologue: lane q < n takes its sample's first draw (held by lane q D),
// loads the first edge and both row bounds, and parks them in the sample's
// record slot (words 0-7 of a 16-byte aligned slot of `stride` words); the
// sample reads them back with read_head before it writes its record there.
__device__ __forceinline__ void prefetch_heads(const DGraph& g, bool oriented, const Draws& dr, int D, int n,
                                               uint32_t* rec, int stride, const LearnArgs* la = nullptr) {
    const int lane = (int)(threadIdx.x & 63);
    const uint32_t rlo = __shfl(dr.lo, lane * D), rhi = __shfl(dr.hi, lane * D);
    if (lane < n) {
        const uint64_t M = oriented ? (uint64_t)g.m : 2ull * (uint64_t)g.m;
        const uint64_t e = __umul64hi(M, ((uint64_t)rhi << 32) | rlo);
        int32_t h0, h1;
        if (oriented) {
            const int2 pr = g.epair[e];
            h0 = pr.x;
            h1 = pr.y;
        } else {
            h0 = g.arow[e];
            h1 = g.nbr[e];
        }
        const int64_t b0 = g.off[h0], e0 = g.off[h0 + 1], b1 = g.off[h1], e1 = g.off[h1 + 1];
        uint4* h4 = reinterpret_cast<uint4*>(rec + lane * stride);
        h4[0] = make_uint4((uint32_t)h0, (uint32_t)h1, (uint32_t)(e0 - b0), (uint32_t)(e1 - b1));
        h4[1] = make_uint4((uint32_t)b0, (uint32_t)((uint64_t)b0 >> 32), (uint32_t)b1, (uint32_t)((uint64_t)b1 >> 32));
        if (la) {  // words 8-9: the buckets of the first edge's ends (learned proposal)
            uint2* k2 = reinterpret_cast<uint2*>(rec + lane * stride + 8);
            k2[0] = make_uint2((uint32_t)bucket_of_degree((int32_t)(e0 - b0)),
                               (uint32_t)bucket_of_degree((int32_t)(e1 - b1)));
        }
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ Head read_head(const uint32_t* slot, bool learned = false) {
    const uint4 a4 = reinterpret_cast<const uint4*>(slot)[0];
    const uint4 b4 = reinterpret_cast<const uint4*>(slot)[1];
    Head h;
    h.k0 = h.k1 = 0;
    if (learned) {
        const uint2 k2 = reinterpret_cast<const uint2*>(slot + 8)[0];
        h.k0 = rfl((int32_t)k2.x);
        h.k1 = rfl((int32_t)k2.y);
    }
    h.v0 = rfl((int32_t)a4.x);
    h.v1 = rfl((int32_t)a4.y);
    h.l0 = rfl((int32_t)a4.z);
    h.l1 = rfl((int32_t)a4.w);
    h.b0 = rfl64((int64_t)(((uint64_t)b4.y << 32) | b4.x));
    h.b1 = rfl64((int64_t)(((uint64_t)b4.w << 32) | b4.z));
    return h;
}

// Whether x is in the ascending row R[0, L), by the whole wave: G-ary rounds
// (64 probes, keep the gap that holds x) until one window of 64 remains.
__device__ __forceinline__ bool wave_row_has(const int32_t* __restrict__ R, int32_t L, int32_t x) {
    const int lane = (int)(threadIdx.x & 63);
    int32_t lo = 0, hi = L;
    while (hi - lo > 64) {
        const int32_t step = (hi - lo) / 64;
        const int32_t pv = R[lo + (lane + 1) * step - 1];
        const int nb = (int)__popcll(__ballot(pv < x));
        if (nb < 64) hi = lo + (nb + 1) * step;
        lo += nb * step;
    }
    const int32_t y = lo + lane < hi ? R[lo + lane] : BIG;
    return __ballot(y == x) != 0ull;
}

// One NS-base sample (lazy verification), one sample per wave: the sampler the
// paper measures NS-prune against (Sec. 4.2).  After the first edge, position
// j is drawn uniformly from the union U_j of the rows of the earlier positions
// joined to j by a pattern edge, enumerated row by row in ascending position,
// each row ascending, an entry kept at its first occurrence; alpha *= |U_j|.
// No other test runs until every position is drawn; the closure check then
// tests distinctness, the symmetry-breaking bounds, every pattern edge and
// (vertex-induced) every non-edge.  Returns 0xFF for a hit, j for an empty
// union at position j, k for a failed closure check.  `list` (CAP words) keeps
// the first CAP members of U_j; a draw beyond them rescans the rows.
template <int KMAX>
__device__ __forceinline__ uint32_t ns_base_sample(const DGraph& g, const Plan& p, uint64_t seed, uint32_t tag,
                                                  uint64_t s, int32_t (&v)[8], uint64_t& alo, uint64_t& ahi,
                                                  uint64_t& ovf, int32_t* list, const Draws* dr) {
    constexpr int CAP = LDS_WORDS / 4;
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = -1;
    const int pk = p.k;
    const uint64_t M = p.oriented ? (uint64_t)g.m : 2ull * (uint64_t)g.m;
    const int32_t* rp[8];
    int32_t rl[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        rp[i] = nullptr;
        rl[i] = 0;
    }
    {
        const uint64_t e = __umul64hi(M, draw_at(dr, seed, s, 0, tag));
        if (p.oriented) {
            const int2 pr = g.epair[e];
            v[0] = pr.x;
            v[1] = pr.y;
        } else {
            v[0] = g.arow[e];
            v[1] = g.nbr[e];
        }
        const int64_t b0 = g.off[v[0]], e0 = g.off[v[0] + 1];
        const int64_t b1 = g.off[v[1]], e1 = g.off[v[1] + 1];
        rp[0] = g.nbr + b0;
        rl[0] = (int32_t)(e0 - b0);
        rp[1] = g.nbr + b1;
        rl[1] = (int32_t)(e1 - b1);
    }
    alo = M;
    ahi = 0;
#pragma unroll
    for (int j = 2; j < KMAX; ++j) {
        if (j >= pk) break;
        const uint32_t conn = (uint32_t)p.connect[j];
        // one chunk of row i: x and whether it is a first occurrence (absent
        // from every earlier joined row); cursors only move forward along row i
        int32_t cur[8];
        auto chunk = [&](int i, int32_t base, int32_t& x) -> bool {
            const bool act = base + lane < rl[i];
            x = act ? rp[i][base + lane] : BIG;
            const uint64_t am = __ballot(act);
            const int32_t xmax = rfl(__shfl(x, (int)__popcll(am) - 1));
            bool fresh = act;
#pragma unroll
            for (int h = 0; h < i; ++h)
                if (conn >> h & 1) {
                    const bool f = member<64>(rp[h], rl[h], cur[h], x, act, xmax, 0, lane, ~0ull);
                    fresh = fresh && !f;
                }
            return fresh;
        };
        // count pass, keeping the first CAP members
        uint64_t cnt = 0;
#pragma unroll
        for (int i = 0; i < KMAX - 1; ++i) {
            if (i >= j || !(conn >> i & 1)) continue;
#pragma unroll
            for (int h = 0; h < 8; ++h) cur[h] = 0;
            for (int32_t base = 0; base < rl[i]; base += 64) {
                int32_t x;
                const bool ok = chunk(i, base, x);
                const uint64_t okm = __ballot(ok);
                const uint64_t rank = (uint64_t)__popcll(okm & below);
                if (ok && cnt + rank < (uint64_t)CAP) list[cnt + rank] = x;
                cnt += (uint64_t)__popcll(okm);
            }
        }
        if (cnt == 0) return (uint32_t)j;
        const uint64_t idx = __umul64hi(cnt, draw_at(dr, seed, s, (uint32_t)j, tag));
        int32_t pick = -1;
        if (idx < (uint64_t)CAP) {
            pick = rfl(list[idx]);
        } else {
            // beyond the kept members: enumerate again up to member idx
            uint64_t seen = 0;
#pragma unroll
            for (int i = 0; i < KMAX - 1; ++i) {
                if (i >= j || !(conn >> i & 1) || pick >= 0) continue;
#pragma unroll
                for (int h = 0; h < 8; ++h) cur[h] = 0;
                for (int32_t base = 0; base < rl[i]; base += 64) {
                    int32_t x;
                    const bool ok = chunk(i, base, x);
                    uint64_t okm = __ballot(ok);
                    const uint64_t c = (uint64_t)__popcll(okm);
                    if (seen + c > idx) {
                        for (uint64_t t = idx - seen; t > 0; --t) okm &= okm - 1ull;
                        pick = rfl(__shfl(x, __ffsll((unsigned long long)okm) - 1));
                        break;
                    }
                    seen += c;
                }
            }
        }
        if (pick < 0) {  // the two passes disagree: report, never index with it
            ovf = 1;
            return (uint32_t)j;
        }
        v[j] = pick;
        if (j + 1 < pk) {
            const int64_t bj = g.off[pick], ej = g.off[pick + 1];
            rp[j] = g.nbr + bj;
            rl[j] = (int32_t)(ej - bj);
        }
        // alpha *= |U_j| with 128-bit overflow detection
        const uint64_t plo = alo * cnt, phi = __umul64hi(alo, cnt);
        const uint64_t qlo = ahi * cnt, qhi = __umul64hi(ahi, cnt);
        const uint64_t nhi = phi + qlo;
        if (qhi != 0 || nhi < qlo) ovf = 1;
        alo = plo;
        ahi = nhi;
    }
    // closure check: what NS-prune tests at every step, tested once at the end
#pragma unroll
    for (int j = 2; j < KMAX; ++j) {
        if (j >= pk) break;
        const uint32_t conn = (uint32_t)p.connect[j], disc = (uint32_t)p.disconnect[j];
        const uint32_t up = (uint32_t)p.upper[j], lw = (uint32_t)p.lower[j];
#pragma unroll
        for (int i = 0; i < KMAX - 1; ++i) {
            if (i >= j) continue;
            if (v[j] == v[i]) return (uint32_t)pk;
            if ((up >> i & 1) && !(v[j] < v[i])) return (uint32_t)pk;
            if ((lw >> i & 1) && !(v[j] > v[i])) return (uint32_t)pk;
        }
#pragma unroll
        for (int i = 0; i < KMAX - 1; ++i) {
            if (i >= j || !((conn | disc) >> i & 1)) continue;
            const bool has = wave_row_has(rp[i], rl[i], v[j]);
            if ((conn >> i & 1) ? !has : has) return (uint32_t)pk;
        }
    }
    return 0xFFu;
}

// Next ticket of a wave from the NTK counters at tk (wave-uniform result).
// Blocks are dispatched round-robin over the 8 XCDs, so starting at counter
// blockIdx % NTK keeps the counters' atomics apart; a wave whose counter has
// run past `ntickets` moves on to the next one and stops after NTK dry
// counters, so every wave ends after at most NTK failed fetches.
__device__ __forceinline__ bool next_ticket(unsigned long long* __restrict__ tk, uint64_t ntickets, int& cur,
                                            int& left, uint64_t& t) {
    while (left > 0) {
        unsigned long long got = 0;
        if ((threadIdx.x & 63) == 0) got = atomicAdd(tk + (size_t)cur * TK_STRIDE, 1ull);
        got = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(__shfl(got, 0) >> 32)) << 32) |
              (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)__shfl(got, 0));
        const uint64_t tt = got * (uint64_t)NTK + (uint64_t)cur;
        if (tt < ntickets) {
            t = tt;
            return true;
        }
        cur = cur + 1 == NTK ? 0 : cur + 1;
        --left;
    }
    return false;
}

// A sample's 16-word LDS record from wave-uniform values, four 16-byte
// stores by one lane: words 0..K-1 the walk, 8 the status, 9-12 the weight
// X (four 32-bit digits), 13-14 the bytes read, 15 zero.  rec is 16-byte aligned.
template <int K>
__device__ __forceinline__ void write_record(uint32_t* rec, const int32_t* v, uint32_t st, uint64_t alo,
                                             uint64_t ahi, uint64_t b) {
    uint4* r4 = reinterpret_cast<uint4*>(rec);
    r4[0] = make_uint4((uint32_t)v[0], (uint32_t)v[1], K > 2 ? (uint32_t)v[2] : 0u, K > 3 ? (uint32_t)v[3] : 0u);
    if (K > 4)
        r4[1] = make_uint4((uint32_t)v[4], K > 5 ? (uint32_t)v[5] : 0u, K > 6 ? (uint32_t)v[6] : 0u,
                           K > 7 ? (uint32_t)v[7] : 0u);
    r4[2] = make_uint4(st, (uint32_t)alo, (uint32_t)(alo >> 32), (uint32_t)ahi);
    r4[3] = make_uint4((uint32_t)(ahi >> 32), (uint32_t)b, (uint32_t)(b >> 32), 0u);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}


}  // namespace sgpm
