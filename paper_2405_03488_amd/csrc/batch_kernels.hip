// Persistent multi-query NS kernel with device-side convergence detection.
//
// Each query keeps the NS-online loop of Sec. 4.1: windows of sample ids
// [n_t, n_{t+1}) and a stop test at every window end.  All queries share one
// launch: waves pull (query, tile) tickets, sample the tile with the query's
// own lane count, add the tile's exact sums into the query's window columns,
// and count finished samples.  The wave whose samples complete a window folds
// the columns into the query's totals, evaluates the predicted error exactly as
// the host does (exact n*S2 - S1^2, correctly rounded conversions, IEEE
// division and square root) and either finishes the query or opens the next
// window by publishing a new epoch in the ticket word (epoch << 40 | tile).
// Window bounds are a deterministic function of the epoch, recomputed by each
// wave, so no wave ever reads bounds another wave is rewriting.  A query's
// samples, sums and stop point are therefore identical to a solo run.
#include "ns_device.h"

namespace sgpm {

namespace {

constexpr unsigned long long TILE_MASK = (1ull << 40) - 1ull;

// Polling reads are relaxed: the words polled (ticket, finished, active) carry
// no data that a wave reads afterwards, and an acquire at agent scope would
// invalidate the XCD's L2, which holds the graph's hot rows.
__device__ __forceinline__ unsigned long long ld_rlx(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_rlx_i(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ uint64_t dev_next_window(uint64_t n_t, const BatchQuery& Q) {
    auto up = [&](uint64_t x) { return Q.quantum ? (x + Q.quantum - 1) / Q.quantum * Q.quantum : x; };
    uint64_t nx;
    if (n_t == 0) {
        nx = up(Q.n_min);
    } else {
        const double gr = ceil(__dmul_rn(Q.growth, (double)n_t));
        uint64_t inc = (uint64_t)gr;
        if (inc < Q.w_min) inc = Q.w_min;
        nx = up(n_t + inc);
    }
    if (Q.max_samples && nx > Q.max_samples) nx = Q.max_samples;
    return nx;
}

// window w = [start, end) of the query's schedule
__device__ void dev_window(const BatchQuery& Q, int w, uint64_t& ws, uint64_t& we) {
    if (Q.mode == SGPM_MODE_FIXED_N) {
        ws = 0;
        we = Q.fixed_n;
        return;
    }
    uint64_t a = 0, b = dev_next_window(0, Q);
    for (int t = 0; t < w; ++t) {
        a = b;
        b = dev_next_window(a, Q);
    }
    ws = a;
    we = b;
}

// correctly rounded double of a little-endian 32-bit digit integer
__device__ double dev_to_double(const uint32_t* d, int nd) {
    int top = -1;
    for (int i = nd - 1; i >= 0; --i)
        if (d[i]) {
            top = i;
            break;
        }
    if (top < 0) return 0.0;
    const int L = 32 * top + 32 - __clz(d[top]);
    auto bit = [&](int i) -> uint32_t { return i < 0 ? 0u : (d[i >> 5] >> (i & 31)) & 1u; };
    if (L <= 64) {
        const uint64_t v = ((uint64_t)(top >= 1 ? d[1] : 0u) << 32) | d[0];
        return (double)v;  // the conversion rounds to nearest even
    }
    const int shift = L - 64;
    uint64_t topbits = 0;
    for (int b = 63; b >= 0; --b) topbits = (topbits << 1) | bit(shift + b);
    bool sticky = false;
    for (int i = 0; i < shift && !sticky; ++i) sticky = bit(i);
    uint64_t keep = topbits >> 11;
    const uint64_t rem = topbits & 0x7FF;
    if (rem > 0x400 || (rem == 0x400 && (sticky || (keep & 1)))) keep++;
    return ldexp((double)keep, shift + 11);
}

// predicted relative error from exact totals (the host's formula and order)
__device__ double dev_eps_hat(double z, uint64_t n, const uint32_t* s1, const uint32_t* s2) {
    bool zero = true;
    for (int i = 0; i < 8; ++i) zero = zero && s1[i] == 0;
    if (n == 0 || zero) return __longlong_as_double(0x7FF0000000000000ll);
    uint32_t D[24], T[24];
    for (int i = 0; i < 24; ++i) D[i] = T[i] = 0;
    const uint32_t N[2] = {(uint32_t)n, (uint32_t)(n >> 32)};
    for (int i = 0; i < 2; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < 12 && i + j < 24; ++j) {
            const uint64_t t = (uint64_t)N[i] * s2[j] + D[i + j] + carry;
            D[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        for (int k = i + 12; k < 24 && carry; ++k) {
            const uint64_t t = (uint64_t)D[k] + carry;
            D[k] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    for (int i = 0; i < 8; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < 8 && i + j < 24; ++j) {
            const uint64_t t = (uint64_t)s1[i] * s1[j] + T[i + j] + carry;
            T[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        for (int k = i + 8; k < 24 && carry; ++k) {
            const uint64_t t = (uint64_t)T[k] + carry;
            T[k] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    int64_t borrow = 0;
    for (int i = 0; i < 24; ++i) {
        const int64_t t = (int64_t)D[i] - (int64_t)T[i] - borrow;
        borrow = t < 0 ? 1 : 0;
        D[i] = (uint32_t)(t & 0xFFFFFFFFll);
    }
    if (borrow) return __longlong_as_double(0x7FF8000000000000ll);
    const double dD = dev_to_double(D, 24), dn = (double)n, dS1 = dev_to_double(s1, 8);
    const double q = __ddiv_rn(dD, dn);
    const double r = __dsqrt_rn(q);
    const double t = __dmul_rn(z, r);
    return __ddiv_rn(t, dS1);
}

// fold the window columns into the totals and decide (one lane)
__device__ __attribute__((noinline)) void complete_window(const BatchQuery& Q, BatchState& S, int w, uint64_t we,
                                unsigned long long* active) {
    unsigned long long col[PF_N];
    for (int i = 0; i < PF_N; ++i) {
        col[i] = 0;
        for (int x = 0; x < 8; ++x)
            col[i] += __hip_atomic_exchange(&S.win[x][i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // S1 columns 0-5 into 8 digits, S2 columns 6-15 into 12 digits
    unsigned long long c = 0;
    for (int i = 0; i < 8; ++i) {
        const unsigned long long t = S.tot_s1[i] + (i < 6 ? col[PF_S1 + i] : 0ull) + c;
        S.tot_s1[i] = t & 0xFFFFFFFFull;
        c = t >> 32;
    }
    c = 0;
    for (int i = 0; i < 12; ++i) {
        const unsigned long long t = S.tot_s2[i] + (i < 10 ? col[PF_S2 + i] : 0ull) + c;
        S.tot_s2[i] = t & 0xFFFFFFFFull;
        c = t >> 32;
    }
    S.hits += col[PF_HITS];
    S.csum += col[PF_CSUM];
    S.bytes += col[PF_BYTES];
    S.ovf += col[PF_OVF];
    S.n = we;
    S.windows = w + 1;
    uint32_t s1[8], s2[12];
    for (int i = 0; i < 8; ++i) s1[i] = (uint32_t)S.tot_s1[i];
    for (int i = 0; i < 12; ++i) s2[i] = (uint32_t)S.tot_s2[i];
    const double eh = dev_eps_hat(Q.z, we, s1, s2);
    S.eps_hat = eh;
    bool stop = false;
    if (S.ovf) {
        stop = true;
        S.status = SGPM_EOVERFLOW;
    } else if (Q.mode == SGPM_MODE_FIXED_N) {
        stop = true;
        S.converged = eh <= Q.eps ? 1 : 0;
    } else if (eh <= Q.eps) {
        stop = true;
        S.converged = 1;
    } else if (Q.max_samples && we >= Q.max_samples) {
        stop = true;
    } else if (dev_next_window(we, Q) <= we) {
        stop = true;
    } else if (w + 1 >= Q.window_cap) {
        stop = true;  // the next window is too large for 64-bit digit columns
        S.status = SGPM_EUNSUPPORTED;
    }
    if (stop) {
        __hip_atomic_store(&S.finished, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        atomicSub(active, 1ull);
    } else {
        __hip_atomic_store(&S.done, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        for (int c = 0; c < 8; ++c)
            __hip_atomic_exchange(&S.ticket[c].v, (unsigned long long)(w + 1) << 40, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }
}

// A wave's sums of one (query, window) are held in LDS as the window columns'
// layout (PF_S1.. 32-bit digit columns of S1, PF_S2.. of S2, PF_HITS,
// PF_CSUM); every sample adds normalised digits (each below 2^32), so a
// column of a window below 2^32 samples cannot wrap.
//
// One tile of samples, one sample per wave at a time, in groups of up to 16
// as in the window kernel: the group's Philox draws are evaluated in parallel
// lanes and read back with readlane, each sample leaves a record in LDS, and
// lane q of the group epilogue hashes record q and adds the digits of X and of
// X^2 to the wave's LDS sums, which the caller adds to the query's window
// columns.
constexpr int BGMAX = 16, BREC = 16;

// CLQ: the query is the KMAX-clique (its compiled plan is the clique's), and the
// sampler is the clique specialisation of the solo kernels
template <int KMAX, bool CLQ>
__device__ __forceinline__ void run_tile(const BatchQuery& Q, uint64_t s0, uint64_t s1, int32_t* list, uint32_t* rec,
                                         unsigned long long* wsum, uint64_t& ovf) {
    const int lane = (int)(threadIdx.x & 63);
    const int K = CLQ ? KMAX : Q.p.k;
    const int D = K - 1;  // draws per sample: 0, 2, .., k-1
    const int GS = (64 / D) < BGMAX ? (64 / D) : BGMAX;
    for (uint64_t gb = s0; gb < s1; gb += (uint64_t)GS) {
        const int n = (int)min((uint64_t)GS, s1 - gb);
        Draws dr;
        {
            const int q = lane / D, t = lane - q * D;
            uint64_t r = 0;
            if (q < n) r = philox_r64(Q.seed, gb + (uint64_t)q, t == 0 ? 0u : (uint32_t)(t + 1), Q.tag);
            dr.lo = (uint32_t)r;
            dr.hi = (uint32_t)(r >> 32);
            dr.k1 = K - 1;
            dr.base = 0;
        }
        prefetch_heads(Q.g, CLQ || Q.p.oriented, dr, D, n, rec, BREC);
        for (int q = 0; q < n; ++q) {
            const uint64_t s = gb + (uint64_t)q;
            dr.base = q * D;
            int32_t v[8];
            uint64_t alo, ahi, b = 0, ov = 0;
            const Head hd = read_head(rec + q * BREC);
            const uint32_t st = ns_sample<64, KMAX, CLQ>(Q.g, Q.p, Q.seed, Q.tag, s, v, alo, ahi, ov, b, false, list,
                                                         nullptr, nullptr, nullptr, &dr, &hd);
            ovf |= ov;
            if (st != 0xFFu) {
                alo = 0;
                ahi = 0;
            }
            // record: 0-7 the walk, 8 the status, 9-12 X
            if (lane == 0) write_record<KMAX>(rec + q * BREC, v, st, alo, ahi, 0);
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < n) {
            const uint32_t* r = rec + lane * BREC;
            const uint32_t st = r[8];
            uint32_t d[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) d[i] = r[9 + i];
            uint64_t h = fmix64((gb + (uint64_t)lane) ^ 0x9E3779B97F4A7C15ull);
            h = fmix64(h ^ (uint64_t)st);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (i < K) h = fmix64(h ^ (uint64_t)r[i]);
            h = fmix64(h ^ ((uint64_t)d[1] << 32 | d[0]));
            h = fmix64(h ^ ((uint64_t)d[3] << 32 | d[2]));
            atomicAdd(&wsum[PF_CSUM], (unsigned long long)h);
            if (st == 0xFFu) {
                uint64_t c2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint64_t pr = (uint64_t)d[a] * (uint64_t)d[e];
                        c2[a + e] += pr & 0xFFFFFFFFull;
                        if (a + e + 1 < 8) c2[a + e + 1] += pr >> 32;
                    }
                // X^2 < 2^256: the columns normalise into 8 digits
                uint64_t cy = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint64_t t = c2[i] + cy;
                    c2[i] = t & 0xFFFFFFFFull;
                    cy = t >> 32;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) atomicAdd(&wsum[PF_S1 + i], (unsigned long long)d[i]);
#pragma unroll
                for (int i = 0; i < 8; ++i) atomicAdd(&wsum[PF_S2 + i], (unsigned long long)c2[i]);
                atomicAdd(&wsum[PF_HITS], 1ull);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// One tile with G lanes per sample (G = 1, 4, 16), as in the solo window
// kernel: group q of the wave takes samples s0 + q, s0 + q + 64/G, ...; its
// leader keeps the exact sums of its samples, and at the tile's end the wave
// adds their 32-bit digits into its LDS sums.
template <int G, int KMAX>
__device__ __forceinline__ void run_tile_g(const BatchQuery& Q, uint64_t s0, uint64_t s1, int32_t* list,
                                           unsigned long long* wsum, uint64_t& ovf) {
    const int lane = (int)(threadIdx.x & 63);
    const bool leader = (lane & (G - 1)) == 0;
    constexpr int CAP = LDS_WORDS / (256 / G);
    int32_t* glist = list + (lane / G) * CAP;
    Acc a;
#pragma unroll
    for (int i = 0; i < 3; ++i) a.s1[i] = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) a.s2[i] = 0;
    a.hits = a.csum = 0;
    for (uint64_t base = s0; base < s1; base += (uint64_t)(64 / G)) {
        const uint64_t s = base + (uint64_t)(lane / G);
        if (s >= s1) break;  // the whole group leaves together
        int32_t v[8];
        uint64_t alo, ahi, b = 0, ov = 0;
        const uint32_t st = ns_sample<G, KMAX>(Q.g, Q.p, Q.seed, Q.tag, s, v, alo, ahi, ov, b, false, glist);
        ovf |= ov;
        if (!leader) continue;
        if (st != 0xFFu) {
            alo = 0;
            ahi = 0;
        } else {
            a.hits += 1;
            acc_add(a, alo, ahi);
        }
        uint64_t h = fmix64(s ^ 0x9E3779B97F4A7C15ull);
        h = fmix64(h ^ (uint64_t)st);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < Q.p.k) h = fmix64(h ^ (uint64_t)(uint32_t)v[i]);
        h = fmix64(h ^ alo);
        h = fmix64(h ^ ahi);
        a.csum += h;
    }
    // the leaders' exact sums as digit columns, summed over the wave
    unsigned long long f[PF_N];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        f[PF_S1 + 2 * i] = a.s1[i] & 0xFFFFFFFFull;
        f[PF_S1 + 2 * i + 1] = a.s1[i] >> 32;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        f[PF_S2 + 2 * i] = a.s2[i] & 0xFFFFFFFFull;
        f[PF_S2 + 2 * i + 1] = a.s2[i] >> 32;
    }
    f[PF_HITS] = a.hits;
    f[PF_CSUM] = a.csum;
#pragma unroll
    for (int i = 0; i < PF_N; ++i) {
        if (i == PF_BYTES || i == PF_OVF) continue;
        const unsigned long long x = wave_sum(f[i]);
        if (lane == 0) wsum[i] += x;
    }
    __builtin_amdgcn_wave_barrier();
}

#ifndef SGPM_BATCH_IDLE_SLEEP
#define SGPM_BATCH_IDLE_SLEEP 8
#endif
#ifndef SGPM_BATCH_WATCHDOG_S
#define SGPM_BATCH_WATCHDOG_S 60
#endif
// blocks per CU the kernel is compiled for: the most at which the sampling
// loops of that pattern bound keep every value in registers (the all-clique
// build inlines one sampler per clique size, so it needs more of them)
// (a build with the lane-group samplers holds a walk per lane in vector
// registers, as the solo window kernel does, and runs at its occupancy)
#ifndef SGPM_BATCH_OCC_CLQ
#define SGPM_BATCH_OCC_CLQ 0  // > 0: waves per SIMD of the all-clique builds
#endif
#ifndef SGPM_BATCH_OCC_GEN
#define SGPM_BATCH_OCC_GEN 0  // > 0: waves per SIMD of the generic builds
#endif
// (all-clique builds for 4 and 5 vertices: 7 waves per SIMD with a few vector
// spills beat 5 without, 10.9 against 12.5 ms for four 4-clique and four
// 5-clique queries to 1 % on R-MAT 20)
constexpr int batch_occupancy(int kmax, bool clq, bool grp) {
    return grp ? 3 : clq ? (SGPM_BATCH_OCC_CLQ > 0 ? SGPM_BATCH_OCC_CLQ : kmax == 4 || kmax == 5 ? 7 : 5)
                       : SGPM_BATCH_OCC_GEN > 0 ? SGPM_BATCH_OCC_GEN : kmax <= 5 ? 6 : kmax == 6 ? 5 : 4;
}

// a tile of a k-clique query (3 <= k <= KMAX) with the sampler compiled for k
template <int KMAX>
__device__ __forceinline__ void clique_tile(int k, const BatchQuery& Q, uint64_t s0, uint64_t s1, int32_t* list,
                                            uint32_t* rec, unsigned long long* wsum, uint64_t& ovf) {
    if (k == KMAX) {
        run_tile<KMAX, true>(Q, s0, s1, list, rec, wsum, ovf);
    } else if constexpr (KMAX > 3) {
        clique_tile<KMAX - 1>(k, Q, s0, s1, list, rec, wsum, ovf);
    }
}

// The wave's sums of one window, held in its LDS columns across tiles, into the
// query's window columns (the copy of this block's XCD: blocks are dispatched
// round-robin over the 8 XCDs, so the copies split the atomics' contention);
// then the held sample count into done, whose last adder completes the window.
__device__ __forceinline__ void flush_held(const BatchQuery* queries, BatchState* states, int hq, int hw,
                                           uint64_t hws, uint64_t hwe, uint64_t hn, uint64_t hovf,
                                           unsigned long long* wsum, unsigned long long* active) {
    const int lane = (int)(threadIdx.x & 63);
    BatchState& S = states[hq];
    unsigned long long* win = S.win[blockIdx.x & 7];
    if (lane < PF_N && lane != PF_BYTES && lane != PF_OVF) {
        const unsigned long long val = wsum[lane];
        wsum[lane] = 0ull;
        if (val) atomicAdd(&win[lane], val);
    }
    if (lane == PF_OVF && hovf) atomicAdd(&win[PF_OVF], (unsigned long long)hovf);
    __builtin_amdgcn_wave_barrier();
    // release only: the sums above before the count below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) {
        const unsigned long long old = atomicAdd(&S.done, (unsigned long long)hn);
        if (old + hn == hwe - hws) {
            __threadfence();
            complete_window(queries[hq], S, hw, hwe, active);
        }
    }
}

// KMAX: the largest pattern size of the batch (the sampler is compiled for it).
// ALLCLQ: every query is a clique of at most KMAX vertices, and each tile runs
// the clique sampler compiled for its query's size.  GRP: some query samples
// with 1, 4 or 16 lanes per sample (its BatchQuery::lanes), and each tile runs
// the sampler of its query's lane count.
//
// Scheduling: a wave takes tiles from the query it served last while that
// query's window has tiles left, trying its own XCD's counter first and the
// other seven after it, then moves on to the next query.  A tile belongs to the
// window the counter's epoch names when the atomic returns it, not to the one
// read before, so a tile handed out across a window change is never lost.  The
// wave keeps its sums in LDS until it moves to another (query, window) or finds
// no tile; a window cannot complete while a wave holds part of it, so every
// wave holding sums of a finished window flushes at its next poll.
template <int KMAX, bool ALLCLQ, bool GRP>
__global__ __launch_bounds__(256, batch_occupancy(KMAX, ALLCLQ, GRP)) void batch_kernel(const BatchQuery* __restrict__ queries, BatchState* __restrict__ states,
                                                    int nq, unsigned long long* __restrict__ active) {
    const int lane = (int)(threadIdx.x & 63);
    const int wid = (int)(threadIdx.x >> 6);
    __shared__ int32_t s_list[LDS_WORDS];
    __shared__ __align__(16) uint32_t s_rec[4][BGMAX * BREC];
    __shared__ unsigned long long s_wsum[4][PF_N];
    unsigned long long* wsum = s_wsum[wid];
    if (lane < PF_N) wsum[lane] = 0ull;
    __builtin_amdgcn_wave_barrier();
    const int wave = rfl((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int xc = (int)(blockIdx.x & 7);
    int start = wave % nq;
    // per-wave cache of the last window looked up: bounds and tile count
    int cq = -1, cw = -1;
    uint64_t cws = 0, cwe = 0, cnt = 0;
    // the (query, window) whose sums the wave holds, and how many samples
    int hq = -1, hw = -1;
    uint64_t hws = 0, hwe = 0, hn = 0, hovf = 0;
    auto lookup = [&](int qq, int e) {
        if (qq != cq || e != cw) {
            dev_window(queries[qq], e, cws, cwe);
            const uint64_t T = (uint64_t)queries[qq].tile;
            cnt = (cwe - cws + T - 1) / T;
            cq = qq;
            cw = e;
        }
    };
    // Watchdog: a wave that has found no tile for SGPM_BATCH_WATCHDOG_S seconds
    // of the 100 MHz real-time counter leaves (holding no sums: it flushed when
    // it first found nothing).  A healthy batch never idles that long -- a wave
    // idles only while other waves finish a window -- so this ends a launch
    // whose invariants broke; the host reports the unfinished queries.
    uint64_t idle_since = 0;
    for (;;) {
        if (hn == 0 && ld_rlx(active) == 0) break;
        int q = -1, w = 0;
        uint64_t t = 0;
        for (int i = 0; i < nq && q < 0; ++i) {
            const int qq = (start + i) % nq;
            if (rfl(ld_rlx_i(&states[qq].finished))) continue;
            for (int j = 0; j < 8; ++j) {
                const int c = (xc + j) & 7;
                unsigned long long* tk = &states[qq].ticket[c].v;
                const unsigned long long cur = (unsigned long long)rfl64((int64_t)ld_rlx(tk));
                lookup(qq, (int)(cur >> 40));
                if ((uint64_t)c + 8ull * (cur & TILE_MASK) >= cnt) continue;
                unsigned long long got = 0;
                if (lane == 0) got = atomicAdd(tk, 1ull);
                got = (unsigned long long)rfl64((int64_t)__shfl(got, 0));
                const int e = (int)(got >> 40);
                lookup(qq, e);
                const uint64_t tile = (uint64_t)c + 8ull * (got & TILE_MASK);
                if (tile >= cnt) continue;
                q = qq;
                w = e;
                t = tile;
                break;
            }
        }
        const bool flush = hn && (q < 0 || q != hq || w != hw);
        if (flush) {
            flush_held(queries, states, hq, hw, hws, hwe, hn, hovf, wsum, active);
            hn = hovf = 0;
        }
        if (q < 0) {
            if (!flush) {
                const uint64_t now = __builtin_amdgcn_s_memrealtime();
                if (idle_since == 0) idle_since = now;
                else if (now - idle_since > (uint64_t)SGPM_BATCH_WATCHDOG_S * 100000000ull) break;
                __builtin_amdgcn_s_sleep(SGPM_BATCH_IDLE_SLEEP);
            }
            start = (start + 1) % nq;
            continue;
        }
        idle_since = 0;
        start = q;
        const BatchQuery& Q = queries[q];
        const uint64_t T = (uint64_t)Q.tile;
        const uint64_t s0 = cws + t * T, s1 = min(s0 + T, cwe);
        uint64_t ovf = 0;
        int32_t* const wl = s_list + wid * (LDS_WORDS / 4);
        if constexpr (GRP) {
            const int lanes = rfl(Q.lanes);
            if (lanes == 1) run_tile_g<1, KMAX>(Q, s0, s1, wl, wsum, ovf);
            else if (lanes == 4) run_tile_g<4, KMAX>(Q, s0, s1, wl, wsum, ovf);
            else if (lanes == 16) run_tile_g<16, KMAX>(Q, s0, s1, wl, wsum, ovf);
            else run_tile<KMAX, false>(Q, s0, s1, wl, s_rec[wid], wsum, ovf);
        } else if constexpr (ALLCLQ) {
            clique_tile<KMAX>(Q.p.k, Q, s0, s1, wl, s_rec[wid], wsum, ovf);
        } else {
            run_tile<KMAX, false>(Q, s0, s1, wl, s_rec[wid], wsum, ovf);
        }
        hq = q;
        hw = w;
        hws = cws;
        hwe = cwe;
        hn += s1 - s0;
        hovf |= ovf;
    }
}

}  // namespace

// the compiled bound for a batch whose largest pattern has k vertices
int batch_kmax(int k) { return k <= 3 ? 3 : k <= 6 ? k : 8; }

int batch_blocks_per_cu(int kmax, bool clq, bool grp) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define SGPM_BATCH_OCC(KK, CC, GG) \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<KK, CC, GG>, 256, 0)
#define SGPM_BATCH_OCC3(KK) \
    if (grp) SGPM_BATCH_OCC(KK, false, true); else if (clq) SGPM_BATCH_OCC(KK, true, false); \
    else SGPM_BATCH_OCC(KK, false, false)
    switch (batch_kmax(kmax)) {
        case 3: SGPM_BATCH_OCC3(3); break;
        case 4: SGPM_BATCH_OCC3(4); break;
        case 5: SGPM_BATCH_OCC3(5); break;
        case 6: SGPM_BATCH_OCC3(6); break;
        default: if (grp) SGPM_BATCH_OCC(8, false, true); else SGPM_BATCH_OCC(8, false, false); break;
    }
#undef SGPM_BATCH_OCC3
#undef SGPM_BATCH_OCC
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

hipError_t launch_batch(const BatchQuery* q, BatchState* s, int nq, unsigned long long* active, int blocks,
                        int kmax, bool clq, bool grp, hipStream_t st) {
#define SGPM_BATCH_LAUNCH(KK, CC, GG) \
    hipLaunchKernelGGL((batch_kernel<KK, CC, GG>), dim3((unsigned)blocks), dim3(256), 0, st, q, s, nq, active)
#define SGPM_BATCH_LAUNCH3(KK) \
    if (grp) SGPM_BATCH_LAUNCH(KK, false, true); else if (clq) SGPM_BATCH_LAUNCH(KK, true, false); \
    else SGPM_BATCH_LAUNCH(KK, false, false)
    switch (batch_kmax(kmax)) {
        case 3: SGPM_BATCH_LAUNCH3(3); break;
        case 4: SGPM_BATCH_LAUNCH3(4); break;
        case 5: SGPM_BATCH_LAUNCH3(5); break;
        case 6: SGPM_BATCH_LAUNCH3(6); break;
        default: if (grp) SGPM_BATCH_LAUNCH(8, false, true); else SGPM_BATCH_LAUNCH(8, false, false); break;
    }
#undef SGPM_BATCH_LAUNCH3
#undef SGPM_BATCH_LAUNCH
    return hipGetLastError();
}

}  // namespace sgpm
