// Graph-sparsification (GS) engine for gfx950: colour sparsification,
// Bernoulli edge sparsification and the plan-driven exact count.
//
// Colour sparsification (Sec. 2.2 subgraph sampling, Sec. 5.2): every vertex
// gets colour floor(c * r / 2^64), r the Philox4x32-10 value of key = seed and
// counter = (v lo, v hi, 0, 0x40000000 | rep); an edge survives when both
// endpoints share a colour.  The sparsified graph G' keeps the vertex ids, so
// it is the disjoint union of the colour classes and counting on G' is
// counting on every class (the paper's partition-parallel search, Sec. 5.4).
// Passes: colours -> per-row kept counts -> exclusive scans -> compaction of
// rows, arc rows and oriented edges.  Rows are streamed once per pass
// (coalesced, 16 lanes per row); colours are one byte per vertex.
//
// Exact count (GS exact search, Sec. 4.4 nested loops): for every first edge
// the nested loops of the same plan NS-prune samples from, enumerating every
// candidate instead of one and counting the last level's candidates.  One wave
// per first edge; the per-level loop state (chunk of 64 candidates, its valid
// mask, merge cursors, walk vertices) lives in LDS so the depth is a runtime
// value.
#include <mutex>

#include "sgpm_internal.h"

namespace sgpm {

namespace {

constexpr int32_t GBIG = 0x7FFFFFFF;

__device__ __forceinline__ uint64_t philox_colour_r64(uint64_t seed, uint64_t v, uint32_t tag) {
    uint32_t c0 = (uint32_t)v, c1 = (uint32_t)(v >> 32), c2 = 0u, c3 = tag;
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

// Largest row length.  Grid-stride over a bounded grid and one atomic per
// block: atomics on one word serialise, so one per wave (16k of them on R-MAT
// 20) cost as much as a full pass over the arcs.
constexpr int MAXDEG_BLOCKS = 1024;
__global__ __launch_bounds__(256) void max_degree_kernel(const int64_t* __restrict__ off, int64_t n,
                                                         unsigned long long* __restrict__ out) {
    unsigned long long d = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long x = (unsigned long long)(off[u + 1] - off[u]);
        d = x > d ? x : d;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(d, o);
        d = t > d ? t : d;
    }
    __shared__ unsigned long long wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = wmax[0];
        for (int i = 1; i < 4; ++i) m = wmax[i] > m ? wmax[i] : m;
        if (m) atomicMax(out, m);
    }
}

__global__ void colour_kernel(int64_t n, uint32_t c, uint64_t seed, uint32_t rep, uint8_t* __restrict__ col) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    col[v] = (uint8_t)__umul64hi((uint64_t)c, philox_colour_r64(seed, (uint64_t)v, 0x40000000u | rep));
}

// Which arcs survive.  Colour sparsification: both endpoints share a colour.
// Bernoulli edge sparsification (Sec. 2.2, the edge-sparsification
// algorithm): edge {a, b}, a > b, survives repetition rep when
// floor(c * r / 2^64) == 0, r the Philox4x32-10 value of key = seed and
// counter = (a, b, 0, 0x20000000 | rep) -- probability 1/c, decided per
// undirected edge, so both arcs agree.
struct KeepRule {
    const uint8_t* col;  // colour sparsification (nullptr: Bernoulli)
    uint64_t seed;
    uint32_t rep, c;
};

template <bool BES>
__device__ __forceinline__ bool keep_arc(const KeepRule& k, int64_t u, uint8_t cu, int32_t w) {
    if constexpr (BES) {
        const uint32_t a = (uint32_t)(u > w ? u : w), b = (uint32_t)(u > w ? w : u);
        const uint64_t r = philox_colour_r64(k.seed, ((uint64_t)b << 32) | a, 0x20000000u | k.rep);
        return __umul64hi((uint64_t)k.c, r) == 0ull;
    } else {
        return k.col[w] == cu;
    }
}

// Arc-parallel sparsification: arcs in CSR order, tiles of ARC_TILE
// consecutive arcs per block (coalesced reads of the arc's row and neighbour,
// no per-row loop, so a hub's row costs what its arcs cost).  Pass 1 counts the
// surviving arcs (and those with w < u, the oriented edges) per tile; after an
// exclusive scan of the tile counts, pass 2 writes every surviving arc at its
// global rank (the order of arcs is kept, so rows stay ascending) and, at each
// row's first arc, the ranks before it; pass 3 turns those into row offsets
// (an empty row takes the offset of the next non-empty one).
constexpr int ARC_TILE = 2048;  // 256 threads x 8

// This thread's arcs of a tile, a_i = t0 + 256 i + threadIdx.x for i < 8, with
// their keep bits (bit i: arc i survives; low: it survives and w < u, an
// oriented edge).  Every load is issued before any is used -- arc rows and
// neighbours, then the colour gathers -- so a wave keeps the whole tile's loads
// in flight instead of one arc's at a time; indexes past the last arc are
// clamped to arc 0, read, and dropped.  prev (nullable): the row of arc a_i - 1.
template <bool BES>
__device__ __forceinline__ void tile_arcs(const DGraph& g, const KeepRule& kr, int64_t t0, int64_t narcs,
                                          int32_t (&u)[ARC_TILE / 256], int32_t (&w)[ARC_TILE / 256],
                                          int32_t* prev, uint32_t& keep, uint32_t& low) {
    constexpr int NA = ARC_TILE / 256;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int64_t a = t0 + i * 256 + (int64_t)threadIdx.x;
        const int64_t ac = a < narcs ? a : 0;
        u[i] = g.arow[ac];
        w[i] = g.nbr[ac];
        if (prev) prev[i] = g.arow[ac > 0 ? ac - 1 : 0];
    }
    uint8_t cu[NA], cw[NA];
    if constexpr (!BES) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            cu[i] = kr.col[u[i]];
            cw[i] = kr.col[w[i]];
        }
    }
    keep = 0;
    low = 0;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int64_t a = t0 + i * 256 + (int64_t)threadIdx.x;
        bool k;
        if constexpr (BES) k = keep_arc<true>(kr, u[i], (uint8_t)0, w[i]);
        else k = cu[i] == cw[i];
        k = k && a < narcs;
        keep |= (uint32_t)k << i;
        low |= (uint32_t)(k && w[i] < u[i]) << i;
    }
}

template <bool BES>
__global__ __launch_bounds__(256) void arc_count_kernel(DGraph g, KeepRule kr, int64_t narcs,
                                                        int64_t* __restrict__ tk, int64_t* __restrict__ tl) {
    const int64_t t0 = (int64_t)blockIdx.x * ARC_TILE;
    int32_t u[ARC_TILE / 256], w[ARC_TILE / 256];
    uint32_t keep, low;
    tile_arcs<BES>(g, kr, t0, narcs, u, w, nullptr, keep, low);
    int k = __popc(keep), l = __popc(low);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        k += __shfl_xor(k, o);
        l += __shfl_xor(l, o);
    }
    __shared__ int sk[4], sl[4];
    if ((threadIdx.x & 63) == 0) {
        sk[threadIdx.x >> 6] = k;
        sl[threadIdx.x >> 6] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tk[blockIdx.x] = (int64_t)(sk[0] + sk[1] + sk[2] + sk[3]);
        tl[blockIdx.x] = (int64_t)(sl[0] + sl[1] + sl[2] + sl[3]);
    }
}

template <bool BES>
__global__ __launch_bounds__(256) void arc_write_kernel(DGraph g, KeepRule kr, int64_t narcs,
                                                        const int64_t* __restrict__ tko,
                                                        const int64_t* __restrict__ tlo, int32_t* __restrict__ nnbr,
                                                        int32_t* __restrict__ narow, int2* __restrict__ nepair,
                                                        int64_t* __restrict__ rstart, int64_t* __restrict__ rlow) {
    constexpr int NA = ARC_TILE / 256;
    const int lane = (int)(threadIdx.x & 63), wid = (int)(threadIdx.x >> 6);
    const uint64_t below = (1ull << lane) - 1ull;
    // surviving arcs and oriented edges per (group of 256 arcs, wave): the rank
    // of an arc in the tile is the count over earlier groups, then over the
    // earlier waves of its group, then over the earlier lanes of its wave
    __shared__ int sk[NA][4], sl[NA][4];
    const int64_t t0 = (int64_t)blockIdx.x * ARC_TILE;
    int32_t uu[NA], ww[NA], pu[NA];
    uint32_t keepm, lowm;
    tile_arcs<BES>(g, kr, t0, narcs, uu, ww, pu, keepm, lowm);
    uint64_t km[NA], lm[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        km[i] = __ballot((keepm >> i) & 1u);
        lm[i] = __ballot((lowm >> i) & 1u);
        if (lane == 0) {
            sk[i][wid] = (int)__popcll(km[i]);
            sl[i][wid] = (int)__popcll(lm[i]);
        }
    }
    __syncthreads();
    int64_t pos = tko[blockIdx.x], lpos = tlo[blockIdx.x];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int64_t a = t0 + i * 256 + (int64_t)threadIdx.x;
        const int32_t u = uu[i], w = ww[i];
        const bool keep = (keepm >> i) & 1u, low = (lowm >> i) & 1u;
        const bool first = a < narcs && (a == 0 || pu[i] != u);
        int kb = 0, lb = 0, kt = 0, lt = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            if (x < wid) {
                kb += sk[i][x];
                lb += sl[i][x];
            }
            kt += sk[i][x];
            lt += sl[i][x];
        }
        const int64_t p = pos + kb + (int64_t)__popcll(km[i] & below);
        const int64_t lp = lpos + lb + (int64_t)__popcll(lm[i] & below);
        if (keep) {
            nnbr[p] = w;
            narow[p] = u;
            if (low) nepair[lp] = make_int2(u, w);
        }
        if (first) {
            rstart[u] = p;
            rlow[u] = lp;
        }
        pos += kt;
        lpos += lt;
    }
}

__global__ void arc_row_offsets_kernel(const int64_t* __restrict__ off, int64_t n, int64_t narcs,
                                       const int32_t* __restrict__ arow, const int64_t* __restrict__ rstart,
                                       const int64_t* __restrict__ rlow, const int64_t* __restrict__ ktot,
                                       const int64_t* __restrict__ ltot, int64_t* __restrict__ noff,
                                       int64_t* __restrict__ neoff) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    const int64_t a = u < n ? off[u] : narcs;
    if (a < narcs) {
        const int32_t v = arow[a];  // the row that owns arc a: u itself, or the next non-empty row
        noff[u] = rstart[v];
        neoff[u] = rlow[v];
    } else {
        noff[u] = *ktot;
        neoff[u] = *ltot;
    }
}

// exclusive scan of int64 counts: out[0..n] with out[n] = total
constexpr int SCAN_TILE = 2048;  // 256 threads x 8

__global__ __launch_bounds__(256) void scan_block_sums(const int64_t* __restrict__ in, int64_t n,
                                                       int64_t* __restrict__ bsum) {
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
    for (int i = 0; i < 8; ++i) {
        const int64_t k = t0 + (int64_t)threadIdx.x * 8 + i;
        if (k < n) s += in[k];
    }
    __shared__ int64_t red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void scan_block_offsets(int64_t* __restrict__ bsum, int64_t nb) {
    // exclusive scan of nb block sums in place by one block
    __shared__ int64_t part[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = (int64_t)threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bsum[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t t = part[i];
            part[i] = run;
            run += t;
        }
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t t = bsum[b];
        bsum[b] = run;
        run += t;
    }
}

__global__ __launch_bounds__(256) void scan_finish(const int64_t* __restrict__ in, int64_t n,
                                                   const int64_t* __restrict__ boff, int64_t* __restrict__ out) {
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t v[8];
    int64_t s = 0;
    for (int i = 0; i < 8; ++i) {
        const int64_t k = t0 + (int64_t)threadIdx.x * 8 + i;
        v[i] = k < n ? in[k] : 0;
        s += v[i];
    }
    __shared__ int64_t part[256];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 256 thread sums
    for (int st = 1; st < 256; st <<= 1) {
        const int64_t add = (int)threadIdx.x >= st ? part[threadIdx.x - st] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = boff[blockIdx.x] + part[threadIdx.x] - s;
    for (int i = 0; i < 8; ++i) {
        const int64_t k = t0 + (int64_t)threadIdx.x * 8 + i;
        if (k < n) out[k] = run;
        run += v[i];
        if (k == n - 1) out[n] = run;
    }
}

// Exclusive scans of two arrays of n <= SCAN_PAIR_MAX entries by one block
// (out[n] = the total): thread i sums a contiguous run of each array, the
// run sums are scanned across the block, then every run is written out.
constexpr int64_t SCAN_PAIR_MAX = 1 << 16;

__global__ __launch_bounds__(1024) void scan_pair_kernel(const int64_t* __restrict__ a, const int64_t* __restrict__ b,
                                                         int64_t n, int64_t* __restrict__ oa, int64_t* __restrict__ ob) {
    __shared__ int64_t pa[1024], pb[1024];
    const int64_t per = (n + 1023) / 1024;
    const int64_t i0 = (int64_t)threadIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    int64_t sa = 0, sb = 0;
    for (int64_t i = i0; i < i1; ++i) {
        sa += a[i];
        sb += b[i];
    }
    pa[threadIdx.x] = sa;
    pb[threadIdx.x] = sb;
    __syncthreads();
    // Hillis-Steele inclusive scan of the run sums
    for (int st = 1; st < 1024; st <<= 1) {
        const int64_t xa = (int)threadIdx.x >= st ? pa[threadIdx.x - st] : 0;
        const int64_t xb = (int)threadIdx.x >= st ? pb[threadIdx.x - st] : 0;
        __syncthreads();
        pa[threadIdx.x] += xa;
        pb[threadIdx.x] += xb;
        __syncthreads();
    }
    int64_t ra = pa[threadIdx.x] - sa, rb = pb[threadIdx.x] - sb;
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t va = a[i], vb = b[i];
        oa[i] = ra;
        ob[i] = rb;
        ra += va;
        rb += vb;
    }
    if (threadIdx.x == 1023) {
        oa[n] = pa[1023];
        ob[n] = pb[1023];
    }
}

// ------------------------------------------------------------------ exact count
__device__ __forceinline__ int32_t grfl(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Lanes [base, base + G) of a wave enumerate the search tree of one first edge
// together (G = 64: the whole wave).  A colour-sparsified graph has rows of a
// few entries, where a whole wave per edge leaves most lanes idle; narrower
// groups keep 64 / G edges in flight per wave.  Every value the helpers return
// is uniform over the group, and control flow is uniform per group.
template <int G>
struct Lanes {
    int sub, base;
    static constexpr unsigned long long full = G == 64 ? ~0ull : (1ull << G) - 1ull;
    __device__ __forceinline__ unsigned long long ballot(bool q) const {
        const unsigned long long b = __ballot(q);
        if constexpr (G == 64) return b;
        else return (b >> base) & full;
    }
    // x of the group's lane i (a whole wave: i is uniform, read by readlane)
    __device__ __forceinline__ int32_t at(int32_t x, int i) const {
        if constexpr (G == 64) return __builtin_amdgcn_readlane(x, i);
        else return __shfl(x, base + i);
    }
};

// membership of each lane's x in an ascending row by a G-entry window merge:
// the window R[c, c + G) is searched by bisection over lanes; c (uniform) only
// moves forward, past entries below the chunk's largest x when it is done
template <int G>
__device__ __forceinline__ bool grp_member(const int32_t* __restrict__ R, int32_t rl, int32_t& c, int32_t x, bool act,
                                           int32_t xmax, const Lanes<G>& ln) {
    bool found = false, pending = act;
    for (;;) {
        const int32_t b = (c + ln.sub < rl) ? R[c + ln.sub] : GBIG;
        const int32_t bmax = ln.at(b, G - 1);
        // entries of the window below x (at most G - 1), kept as the lane
        // permute's byte address of the group's lane base + pos
        int pb = ln.base * 4;
#pragma unroll
        for (int st = G / 2; st >= 1; st >>= 1) {
            const int32_t bv = __builtin_amdgcn_ds_bpermute(pb + (st - 1) * 4, b);
            pb += bv < x ? st * 4 : 0;
        }
        const int32_t bq = __builtin_amdgcn_ds_bpermute(pb, b);
        const bool res = pending && x <= bmax;
        if (res) found = bq == x;
        pending = pending && !res;
        if (ln.ballot(pending) == 0) {
            c += (int32_t)__popcll(ln.ballot(b < xmax));
            break;
        }
        c += G;
    }
    return found;
}

// plan masks packed 8 bits per position, indexable by a runtime position
struct PackedPlan {
    uint64_t connect, disconnect, upper, lower;
    int32_t k, oriented;
};
__device__ __forceinline__ uint32_t pk(uint64_t m, int j) { return (uint32_t)(m >> (8 * j)) & 0xFFu; }

template <int G>
struct Level {          // per-group, per-level loop state (LDS)
    int32_t base;       // next chunk start in the driver row
    int32_t ended;      // the driver window is exhausted
    int32_t d;          // driver position
    int32_t lo, hi;     // bounds
    uint32_t pad;
    unsigned long long mask;  // unvisited candidates of the current chunk
    int32_t cur[8];     // merge cursors per constraint row
    int32_t xs[G];      // current chunk's values
};

template <int G>
struct GroupState {
    int32_t v[8];
    int64_t rb[8];
    int32_t rl[8];
    Level<G> lv[6];     // levels 2 .. 7
};

// Evaluate the next chunk of level j's candidates; returns the valid mask and
// stores the chunk in L.xs.
template <int G>
__device__ __forceinline__ unsigned long long eval_level_chunk(const DGraph& g, const PackedPlan& p, int j,
                                                               GroupState<G>& W, Level<G>& L, const Lanes<G>& ln,
                                                               int32_t& x_out) {
    const uint32_t conn = pk(p.connect, j), disc = pk(p.disconnect, j);
    const int32_t* dp = g.nbr + W.rb[L.d];
    const int32_t dl = W.rl[L.d];
    const int32_t pos = L.base + ln.sub;
    const int32_t x = pos < dl ? dp[pos] : GBIG;
    const bool act = x < L.hi;
    const unsigned long long inm = ln.ballot(act);  // a prefix of the group
    bool ok = act && x > L.lo;
    for (int i = 0; i < j; ++i)
        if (!(conn >> i & 1)) ok = ok && x != W.v[i];
    if (inm != 0) {
        const int32_t xmax = ln.at(x, (int)__popcll(inm) - 1);
        for (int i = 0; i < j; ++i) {
            const bool isc = (conn >> i & 1) && i != L.d, isd = disc >> i & 1;
            if (!isc && !isd) continue;
            int32_t c = L.cur[i];
            const bool f = grp_member<G>(g.nbr + W.rb[i], W.rl[i], c, x, act, xmax, ln);
            L.cur[i] = c;  // uniform: every lane of the group stores the same value
            ok = ok && (isc ? f : !f);
        }
    }
    if (inm != Lanes<G>::full) L.ended = 1;
    L.base += G;
    x_out = x;
    return ln.ballot(ok);
}

template <int G>
__device__ __forceinline__ void init_level(const DGraph& g, const PackedPlan& p, int j, GroupState<G>& W,
                                           Level<G>& L) {
    const uint32_t conn = pk(p.connect, j), up = pk(p.upper, j), lw = pk(p.lower, j);
    int32_t lo = -1, hi = GBIG, d = -1, dl = GBIG;
    for (int i = 0; i < j; ++i) {
        if (up >> i & 1) hi = min(hi, W.v[i]);
        if (lw >> i & 1) lo = max(lo, W.v[i]);
        if ((conn >> i & 1) && W.rl[i] < dl) {
            d = i;
            dl = W.rl[i];
        }
    }
    int32_t start = 0;
    if (lo >= 0) {
        const int32_t* dp = g.nbr + W.rb[d];
        int32_t a = 0, b = dl;
        while (a < b) {
            const int32_t mid = (a + b) >> 1;
            if (dp[mid] < lo + 1) a = mid + 1;
            else b = mid;
        }
        start = a;
    }
    // uniform values: every lane of the group stores the same, so each lane's
    // later reads follow its own writes in program order
    L.base = start;
    L.ended = 0;
    L.d = d;
    L.lo = lo;
    L.hi = hi;
    L.mask = 0;
    for (int i = 0; i < 8; ++i) L.cur[i] = 0;
}

template <int G>
__global__ __launch_bounds__(256) void exact_count_kernel(DGraph g, PackedPlan p, uint64_t nfirst, TicketPlan tp,
                                                          unsigned long long* __restrict__ ticket,
                                                          unsigned long long* __restrict__ partials,
                                                          const uint32_t* __restrict__ elist) {
    constexpr int NG = 64 / G;  // groups per wave
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const int grp = lane / G;
    const Lanes<G> ln{lane % G, grp * G};
    __shared__ GroupState<G> ws[4 * NG];
    GroupState<G>& W = ws[w * NG + grp];
    unsigned long long total = 0;  // uniform over the group
    const int k = p.k;
    for (;;) {
        unsigned long long t = 0;
        if (ln.sub == 0) t = atomicAdd(ticket, 1ull);
        t = __shfl(t, ln.base);
        if (t >= nfirst) break;
        const uint64_t e0 = ticket_start(tp, t);
        if (e0 >= nfirst) break;
        const uint64_t e1 = min(ticket_start(tp, t + 1), nfirst);
        for (uint64_t ei = e0; ei < e1; ++ei) {
            // first edge ei, or the ei-th of a list of first edges
            const uint64_t e = elist ? (uint64_t)elist[ei] : ei;
            int32_t v0, v1;
            if (p.oriented) {
                const int2 pr = g.epair[e];
                v0 = pr.x;
                v1 = pr.y;
            } else {
                v0 = g.arow[e];
                v1 = g.nbr[e];
            }
            if (k == 2) {
                total += 1;
                continue;
            }
            {
                const int64_t b0 = g.off[v0], b1 = g.off[v1];
                const int32_t l0 = (int32_t)(g.off[v0 + 1] - b0), l1 = (int32_t)(g.off[v1 + 1] - b1);
                W.v[0] = v0;
                W.v[1] = v1;
                W.rb[0] = b0;
                W.rl[0] = l0;
                W.rb[1] = b1;
                W.rl[1] = l1;
            }
            __builtin_amdgcn_wave_barrier();
            int j = 2;
            init_level<G>(g, p, 2, W, W.lv[0]);
            __builtin_amdgcn_wave_barrier();
            while (j >= 2) {
                Level<G>& L = W.lv[j - 2];
                if (j == k - 1) {
                    // last level: count every candidate
                    while (!L.ended) {
                        int32_t x;
                        const unsigned long long okm = eval_level_chunk<G>(g, p, j, W, L, ln, x);
                        __builtin_amdgcn_wave_barrier();
                        total += (unsigned long long)__popcll(okm);
                    }
                    --j;
                    continue;
                }
                if (L.mask == 0) {
                    if (L.ended) {
                        --j;
                        continue;
                    }
                    int32_t x;
                    const unsigned long long okm = eval_level_chunk<G>(g, p, j, W, L, ln, x);
                    L.xs[ln.sub] = x;
                    L.mask = okm;
                    __builtin_amdgcn_wave_barrier();
                    continue;
                }
                const unsigned long long m = L.mask;
                const int bit = __ffsll(m) - 1;
                int32_t vj = L.xs[bit];
                if constexpr (G == 64) vj = grfl(vj);
                {
                    const int64_t bj = g.off[vj];
                    const int32_t lj = (int32_t)(g.off[vj + 1] - bj);
                    L.mask = m & (m - 1ull);
                    W.v[j] = vj;
                    W.rb[j] = bj;
                    W.rl[j] = lj;
                }
                __builtin_amdgcn_wave_barrier();
                ++j;
                init_level<G>(g, p, j, W, W.lv[j - 2]);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __shared__ unsigned long long red[4 * NG];
    if (ln.sub == 0) red[w * NG + grp] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        // two 32-bit halves so the final sum is exact in 64-bit words
        unsigned long long lo = 0, hi = 0;
        for (int i = 0; i < 4 * NG; ++i) {
            lo += red[i] & 0xFFFFFFFFull;
            hi += red[i] >> 32;
        }
        partials[2 * blockIdx.x] = lo;
        partials[2 * blockIdx.x + 1] = hi;
    }
}

// Clique counts (k = 4, 5, 6) by bitmaps over the first edge's candidate set.
// The k-clique plan orders v0 > v1 > ... > v_{k-1}, every later vertex adjacent
// to all earlier ones, so with S = N(v0) ∩ N(v1) ∩ [0, v1) in ascending order
// the tuples through the first edge (v0, v1) are the (k-2)-cliques of the graph
// induced on S, each once in descending order.  One wave per first edge: S
// goes to LDS (at most 64 members; a first edge with a larger S is appended to
// `overflow` for the general search); a window merge of S against the row of
// its member a gives the bitmap M[a] of the members below a adjacent to it;
// the count is sum_a |M[a]| (k = 4), sum_a sum_{b in M[a]} |M[a] & M[b]|
// (k = 5), or one more level (k = 6).  Levels beyond the third cost popcounts
// instead of row merges.
constexpr int CLQ_SET = 64;

template <int KC>
__global__ __launch_bounds__(256) void clique_bitmap_kernel(DGraph g, uint64_t nfirst, TicketPlan tp,
                                                            unsigned long long* __restrict__ ticket,
                                                            unsigned long long* __restrict__ partials,
                                                            uint32_t* __restrict__ overflow,
                                                            unsigned long long* __restrict__ noverflow) {
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const Lanes<64> ln{lane, 0};
    __shared__ int32_t s_set[4][CLQ_SET];
    __shared__ unsigned long long s_mask[4][CLQ_SET];
    int32_t* S = s_set[w];
    unsigned long long* M = s_mask[w];
    unsigned long long total = 0;  // per lane
    for (;;) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(ticket, 1ull);
        t = ((unsigned long long)(uint32_t)grfl((int32_t)(__shfl(t, 0) >> 32)) << 32) |
            (uint32_t)grfl((int32_t)__shfl(t, 0));
        if (t >= nfirst) break;
        const uint64_t e0 = ticket_start(tp, t);
        if (e0 >= nfirst) break;
        const uint64_t e1 = min(ticket_start(tp, t + 1), nfirst);
        for (uint64_t e = e0; e < e1; ++e) {
            const int2 pr = g.epair[e];
            const int32_t v0 = grfl(pr.x), v1 = grfl(pr.y);
            const int64_t b0 = g.off[v0], b1 = g.off[v1];
            const int32_t l0 = (int32_t)(g.off[v0 + 1] - b0), l1 = (int32_t)(g.off[v1 + 1] - b1);
            // S: the shorter row's entries below v1 that the other row holds
            const bool d0 = l0 <= l1;
            const int32_t* dp = g.nbr + (d0 ? b0 : b1);
            const int32_t* op = g.nbr + (d0 ? b1 : b0);
            const int32_t dl = d0 ? l0 : l1, ol = d0 ? l1 : l0;
            int32_t s = 0, cur = 0;
            bool over = false;
            for (int32_t base = 0; base < dl; base += 64) {
                const int32_t x = base + lane < dl ? dp[base + lane] : GBIG;
                const bool act = x < v1;
                const unsigned long long inm = __ballot(act);  // a prefix of the wave
                if (inm == 0) break;
                const int32_t xmax = ln.at(x, (int)__popcll(inm) - 1);
                const bool f = grp_member<64>(op, ol, cur, x, act, xmax, ln);
                const unsigned long long okm = __ballot(act && f);
                const int c = (int)__popcll(okm);
                if (s + c > CLQ_SET) {
                    over = true;
                    break;
                }
                if (act && f) S[s + (int)__popcll(okm & ((1ull << lane) - 1ull))] = x;
                s += c;
                if (inm != ~0ull) break;
            }
            if (over) {
                if (lane == 0) overflow[atomicAdd(noverflow, 1ull)] = (uint32_t)e;
                continue;
            }
            if (s < KC - 2) continue;
            __builtin_amdgcn_wave_barrier();
            const int32_t xs = lane < s ? S[lane] : GBIG;  // ascending over the lanes
            // lane ia: M[ia] = members below S[ia] adjacent to it
            unsigned long long mine = 0;
            for (int ia = 1; ia < s; ++ia) {
                const int32_t a = ln.at(xs, ia);
                const int64_t ba = g.off[a];
                const int32_t la = (int32_t)(g.off[a + 1] - ba);
                int32_t ca = 0;
                const bool act = lane < ia;
                const bool f = grp_member<64>(g.nbr + ba, la, ca, xs, act, ln.at(xs, ia - 1), ln);
                const unsigned long long m = __ballot(act && f);
                if (lane == ia) mine = m;
            }
            M[lane] = mine;
            __builtin_amdgcn_wave_barrier();
            unsigned long long cnt = 0;
            if constexpr (KC == 4) {
                cnt = (unsigned long long)__popcll(mine);
            } else {
                unsigned long long m = mine;
                while (m) {
                    const int b = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1ull;
                    const unsigned long long m2 = mine & M[b];
                    if constexpr (KC == 5) {
                        cnt += (unsigned long long)__popcll(m2);
                    } else {
                        unsigned long long r = m2;
                        while (r) {
                            const int c3 = __ffsll((unsigned long long)r) - 1;
                            r &= r - 1ull;
                            cnt += (unsigned long long)__popcll(m2 & M[c3]);
                        }
                    }
                }
            }
            total += cnt;
            __builtin_amdgcn_wave_barrier();  // S and M are rewritten by the next first edge
        }
    }
    // block sum as the general count's: two 32-bit halves per block
    unsigned long long lo = total & 0xFFFFFFFFull, hi = total >> 32;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo += __shfl_xor(lo, o);
        hi += __shfl_xor(hi, o);
    }
    __shared__ unsigned long long red[4][2];
    if (lane == 0) {
        red[w][0] = lo;
        red[w][1] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
        partials[2 * blockIdx.x + 1] = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    }
}

// The same count for first edges whose candidate set S holds 65 to 128
// members (the 64-member kernel's overflow list): S in two halves of 64 lanes,
// each member's adjacency inside S as a two-word mask, one merge of the row of
// member a against both halves (ascending, so the merge cursor carries from
// the first half into the second).  A set past 128 members is appended to
// `overflow` for the general search.
constexpr int CLQ_SET2 = 128;

template <int KC>
__global__ __launch_bounds__(256) void clique_bitmap128_kernel(DGraph g, const uint32_t* __restrict__ elist,
                                                               uint64_t nlist, TicketPlan tp,
                                                               unsigned long long* __restrict__ ticket,
                                                               unsigned long long* __restrict__ partials,
                                                               uint32_t* __restrict__ overflow,
                                                               unsigned long long* __restrict__ noverflow) {
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const Lanes<64> ln{lane, 0};
    __shared__ int32_t s_set[4][CLQ_SET2];
    __shared__ unsigned long long s_m0[4][CLQ_SET2], s_m1[4][CLQ_SET2];
    int32_t* S = s_set[w];
    unsigned long long* M0 = s_m0[w];
    unsigned long long* M1 = s_m1[w];
    unsigned long long total = 0;  // per lane
    for (;;) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(ticket, 1ull);
        t = ((unsigned long long)(uint32_t)grfl((int32_t)(__shfl(t, 0) >> 32)) << 32) |
            (uint32_t)grfl((int32_t)__shfl(t, 0));
        if (t >= nlist) break;
        const uint64_t e0 = ticket_start(tp, t);
        if (e0 >= nlist) break;
        const uint64_t e1 = min(ticket_start(tp, t + 1), nlist);
        for (uint64_t ei = e0; ei < e1; ++ei) {
            const uint32_t e = (uint32_t)grfl((int32_t)elist[ei]);
            const int2 pr = g.epair[e];
            const int32_t v0 = grfl(pr.x), v1 = grfl(pr.y);
            const int64_t b0 = g.off[v0], b1 = g.off[v1];
            const int32_t l0 = (int32_t)(g.off[v0 + 1] - b0), l1 = (int32_t)(g.off[v1 + 1] - b1);
            const bool d0 = l0 <= l1;
            const int32_t* dp = g.nbr + (d0 ? b0 : b1);
            const int32_t* op = g.nbr + (d0 ? b1 : b0);
            const int32_t dl = d0 ? l0 : l1, ol = d0 ? l1 : l0;
            int32_t s = 0, cur = 0;
            bool over = false;
            for (int32_t base = 0; base < dl; base += 64) {
                const int32_t x = base + lane < dl ? dp[base + lane] : GBIG;
                const bool act = x < v1;
                const unsigned long long inm = __ballot(act);  // a prefix of the wave
                if (inm == 0) break;
                const int32_t xmax = ln.at(x, (int)__popcll(inm) - 1);
                const bool f = grp_member<64>(op, ol, cur, x, act, xmax, ln);
                const unsigned long long okm = __ballot(act && f);
                const int c = (int)__popcll(okm);
                if (s + c > CLQ_SET2) {
                    over = true;
                    break;
                }
                if (act && f) S[s + (int)__popcll(okm & ((1ull << lane) - 1ull))] = x;
                s += c;
                if (inm != ~0ull) break;
            }
            if (over) {
                if (lane == 0) overflow[atomicAdd(noverflow, 1ull)] = e;
                continue;
            }
            if (s < KC - 2) continue;
            __builtin_amdgcn_wave_barrier();
            // ascending over lane and then over 64 + lane
            const int32_t xs0 = lane < s ? S[lane] : GBIG, xs1 = 64 + lane < s ? S[64 + lane] : GBIG;
            // member lane: (lo0, lo1), member 64 + lane: (hi0, hi1)
            unsigned long long lo0 = 0, lo1 = 0, hi0 = 0, hi1 = 0;
            for (int ia = 1; ia < s; ++ia) {
                const int32_t a = ia < 64 ? ln.at(xs0, ia) : ln.at(xs1, ia - 64);
                const int64_t ba = g.off[a];
                const int32_t la = (int32_t)(g.off[a + 1] - ba);
                int32_t ca = 0;
                const int n0 = ia < 64 ? ia : 64;  // members below a in the first half
                const bool act0 = lane < n0;
                const bool f0 = grp_member<64>(g.nbr + ba, la, ca, xs0, act0, ln.at(xs0, n0 - 1), ln);
                const unsigned long long m0 = __ballot(act0 && f0);
                unsigned long long m1 = 0;
                if (ia > 64) {
                    const bool act1 = lane < ia - 64;
                    const bool f1 = grp_member<64>(g.nbr + ba, la, ca, xs1, act1, ln.at(xs1, ia - 65), ln);
                    m1 = __ballot(act1 && f1);
                }
                if (ia < 64) {
                    if (lane == ia) {
                        lo0 = m0;
                        lo1 = m1;
                    }
                } else if (lane == ia - 64) {
                    hi0 = m0;
                    hi1 = m1;
                }
            }
            M0[lane] = lo0;
            M1[lane] = lo1;
            M0[64 + lane] = hi0;
            M1[64 + lane] = hi1;
            __builtin_amdgcn_wave_barrier();
            unsigned long long cnt = 0;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const unsigned long long a0 = half ? hi0 : lo0, a1 = half ? hi1 : lo1;
                if constexpr (KC == 4) {
                    cnt += (unsigned long long)(__popcll(a0) + __popcll(a1));
                } else {
#pragma unroll
                    for (int wd = 0; wd < 2; ++wd) {
                        unsigned long long m = wd ? a1 : a0;
                        while (m) {
                            const int b = (__ffsll((unsigned long long)m) - 1) + 64 * wd;
                            m &= m - 1ull;
                            const unsigned long long c0 = a0 & M0[b], c1 = a1 & M1[b];
                            if constexpr (KC == 5) {
                                cnt += (unsigned long long)(__popcll(c0) + __popcll(c1));
                            } else {
#pragma unroll
                                for (int wd2 = 0; wd2 < 2; ++wd2) {
                                    unsigned long long r = wd2 ? c1 : c0;
                                    while (r) {
                                        const int c3 = (__ffsll((unsigned long long)r) - 1) + 64 * wd2;
                                        r &= r - 1ull;
                                        cnt += (unsigned long long)(__popcll(c0 & M0[c3]) + __popcll(c1 & M1[c3]));
                                    }
                                }
                            }
                        }
                    }
                }
            }
            total += cnt;
            __builtin_amdgcn_wave_barrier();  // S and the masks are rewritten by the next first edge
        }
    }
    unsigned long long lo = total & 0xFFFFFFFFull, hi = total >> 32;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo += __shfl_xor(lo, o);
        hi += __shfl_xor(hi, o);
    }
    __shared__ unsigned long long red[4][2];
    if (lane == 0) {
        red[w][0] = lo;
        red[w][1] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
        partials[2 * blockIdx.x + 1] = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    }
}

// Per-edge terms of the 4-vertex counts that have closed forms over edges
// (each identity is one the oracle's counts are pinned against): with t the
// edge's common neighbours and du, dw its endpoints' degrees, the oriented
// edge list (each edge once) gives
//   ET_DIAMOND  C(t, 2)                      diamonds (one middle edge each)
//   ET_TAILED   t (du + dw - 4)              twice the tailed triangles
//   ET_PATH4    (du - 1)(dw - 1) - t         4-paths (by their middle edge)
//   ET_STAR3    C(du - 1, 2) + C(dw - 1, 2)  three times the 3-stars
//   ET_WEDGE    du + dw - 2                  twice the wedges
//   ET_IWEDGE   du + dw - 2 - 2t             twice the induced wedges
// Every term is below 2^63.  The launch sums the terms sel[0..2] (-1: none);
// a lane adds each term's low and high 32-bit halves separately and every
// block writes its six sums to partials[6 block ..].  With NEED_T the G lanes
// of a group intersect the edge's rows (the shorter row, G entries at a time,
// merged against the longer by the window search); without it (degree terms
// only) every lane takes its own edges.
enum { ET_DIAMOND, ET_TAILED, ET_PATH4, ET_STAR3, ET_WEDGE, ET_IWEDGE };

__device__ __forceinline__ unsigned long long edge_term(int q, unsigned long long t, unsigned long long du,
                                                        unsigned long long dw) {
    switch (q) {
        case ET_DIAMOND: return t * (t - 1ull) / 2ull;  // 0 for t = 0 in unsigned arithmetic
        case ET_TAILED: return t == 0ull ? 0ull : t * (du + dw - 4ull);  // t >= 1: du, dw >= 2
        case ET_PATH4: return (du - 1ull) * (dw - 1ull) - t;
        case ET_STAR3:
            return (du >= 3ull ? (du - 1ull) * (du - 2ull) / 2ull : 0ull) +
                   (dw >= 3ull ? (dw - 1ull) * (dw - 2ull) / 2ull : 0ull);
        case ET_WEDGE: return du + dw - 2ull;
        case ET_IWEDGE: return du + dw - 2ull - 2ull * t;
        default: return 0ull;
    }
}

template <int G, bool NEED_T>
__global__ __launch_bounds__(256) void edge_terms_kernel(DGraph g, TicketPlan tp, int sel0, int sel1, int sel2,
                                                         unsigned long long* __restrict__ ticket,
                                                         unsigned long long* __restrict__ partials) {
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const Lanes<G> ln{lane % G, (lane / G) * G};
    const uint64_t nedges = (uint64_t)g.m;
    const int sel[3] = {sel0, sel1, sel2};
    unsigned long long acc[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};  // (low, high) per selected term
    auto add = [&](unsigned long long t, unsigned long long du, unsigned long long dw) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const unsigned long long v = edge_term(sel[k], t, du, dw);
            acc[2 * k] += v & 0xFFFFFFFFull;
            acc[2 * k + 1] += v >> 32;
        }
    };
    if constexpr (!NEED_T) {
        for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges;
             e += (uint64_t)gridDim.x * blockDim.x) {
            const int2 pr = g.epair[e];
            add(0ull, (unsigned long long)(g.off[pr.x + 1] - g.off[pr.x]),
                (unsigned long long)(g.off[pr.y + 1] - g.off[pr.y]));
        }
    } else {
        for (;;) {
            unsigned long long t = 0;
            if (ln.sub == 0) t = atomicAdd(ticket, 1ull);
            t = __shfl(t, ln.base);
            if (t >= nedges) break;
            const uint64_t e0 = ticket_start(tp, t);
            if (e0 >= nedges) break;
            const uint64_t e1 = min(ticket_start(tp, t + 1), nedges);
            for (uint64_t e = e0; e < e1; ++e) {
                const int2 pr = g.epair[e];
                const int64_t b0 = g.off[pr.x], b1 = g.off[pr.y];
                const int32_t l0 = (int32_t)(g.off[pr.x + 1] - b0), l1 = (int32_t)(g.off[pr.y + 1] - b1);
                const bool d0 = l0 <= l1;
                const int32_t* dp = g.nbr + (d0 ? b0 : b1);
                const int32_t* op = g.nbr + (d0 ? b1 : b0);
                const int32_t dl = d0 ? l0 : l1, ol = d0 ? l1 : l0;
                int32_t cur = 0;
                unsigned long long tc = 0;
                for (int32_t base = 0; base < dl; base += G) {
                    const bool act = base + ln.sub < dl;
                    const int32_t x = act ? dp[base + ln.sub] : GBIG;
                    const int32_t xmax = ln.at(x, min(G, dl - base) - 1);
                    const bool f = grp_member<G>(op, ol, cur, x, act, xmax, ln);
                    tc += (unsigned long long)__popcll(ln.ballot(act && f));
                }
                // every lane of the group holds the same values; its first adds them
                if (ln.sub == 0) add(tc, (unsigned long long)l0, (unsigned long long)l1);
            }
        }
    }
    __shared__ unsigned long long red[4][6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        unsigned long long a = acc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
        if (lane == 0) red[w][k] = a;
    }
    __syncthreads();
    if (threadIdx.x < 6)
        partials[6 * (size_t)blockIdx.x + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// out[k] = sum over the blocks of partials[6 block + k], k < 6
__global__ void sum_six_kernel(const unsigned long long* __restrict__ partials, int nblocks,
                               unsigned long long* __restrict__ out) {
    __shared__ unsigned long long a[6][256];
    unsigned long long s[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    for (int i = (int)threadIdx.x; i < nblocks; i += (int)blockDim.x)
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] += partials[6 * (size_t)i + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k][threadIdx.x] = s[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        unsigned long long t = 0;
        for (int i = 0; i < 256; ++i) t += a[threadIdx.x][i];
        out[threadIdx.x] = t;
    }
}

__global__ void sum_pairs_kernel(const unsigned long long* __restrict__ partials, int nblocks,
                                 unsigned long long* __restrict__ out2) {
    __shared__ unsigned long long a[256], b[256];
    unsigned long long lo = 0, hi = 0;
    for (int i = (int)threadIdx.x; i < nblocks; i += (int)blockDim.x) {
        lo += partials[2 * i];
        hi += partials[2 * i + 1];
    }
    a[threadIdx.x] = lo;
    b[threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long L = 0, H = 0;
        for (int i = 0; i < 256; ++i) {
            L += a[i];
            H += b[i];
        }
        out2[0] = L;  // sum of low halves
        out2[1] = H;  // sum of high halves (weight 2^32)
    }
}

}  // namespace

hipError_t gs_colours(int64_t n, uint32_t c, uint64_t seed, uint32_t rep, uint8_t* col, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(colour_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, c, seed, rep, col);
    return hipGetLastError();
}

int64_t arc_tiles(int64_t narcs) { return (narcs + ARC_TILE - 1) / ARC_TILE; }

// pass 1: per-tile counts of surviving arcs and oriented edges (tk, tl: arc_tiles entries)
hipError_t gs_arc_counts(const DGraph& g, const uint8_t* col, uint32_t c, uint64_t seed, uint32_t rep, int64_t* tk,
                         int64_t* tl, hipStream_t st) {
    const int64_t narcs = 2 * g.m, nt = arc_tiles(narcs);
    if (nt == 0) return hipSuccess;
    const KeepRule kr{col, seed, rep, c};
    if (col) hipLaunchKernelGGL(arc_count_kernel<false>, dim3((unsigned)nt), dim3(256), 0, st, g, kr, narcs, tk, tl);
    else hipLaunchKernelGGL(arc_count_kernel<true>, dim3((unsigned)nt), dim3(256), 0, st, g, kr, narcs, tk, tl);
    return hipGetLastError();
}

// passes 2 and 3: tko, tlo the exclusive scans of the tile counts (arc_tiles + 1
// entries each, the last ones the totals); rstart, rlow n words of scratch;
// noff, neoff n + 1 offsets of the new rows and oriented edges
hipError_t gs_arc_write(const DGraph& g, const uint8_t* col, uint32_t c, uint64_t seed, uint32_t rep,
                        const int64_t* tko, const int64_t* tlo, int32_t* nnbr, int32_t* narow,
                        int2* nepair, int64_t* rstart, int64_t* rlow, int64_t* noff, int64_t* neoff,
                        hipStream_t st) {
    const int64_t narcs = 2 * g.m, nt = arc_tiles(narcs);
    const KeepRule kr{col, seed, rep, c};
    if (nt > 0) {
        if (col)
            hipLaunchKernelGGL(arc_write_kernel<false>, dim3((unsigned)nt), dim3(256), 0, st, g, kr, narcs, tko, tlo,
                               nnbr, narow, nepair, rstart, rlow);
        else
            hipLaunchKernelGGL(arc_write_kernel<true>, dim3((unsigned)nt), dim3(256), 0, st, g, kr, narcs, tko, tlo,
                               nnbr, narow, nepair, rstart, rlow);
    }
    hipLaunchKernelGGL(arc_row_offsets_kernel, dim3((unsigned)((g.n + 1 + 255) / 256)), dim3(256), 0, st, g.off, g.n,
                       narcs, g.arow, rstart, rlow, tko + nt, tlo + nt, noff, neoff);
    return hipGetLastError();
}

hipError_t max_degree(const int64_t* off, int64_t n, unsigned long long* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, MAXDEG_BLOCKS);
    hipLaunchKernelGGL(max_degree_kernel, dim3((unsigned)blocks), dim3(256), 0, st, off, n, out);
    return hipGetLastError();
}

int64_t scan_scratch_words(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t exclusive_scan_pair(const int64_t* a, const int64_t* b, int64_t n, int64_t* oa, int64_t* ob,
                               int64_t* scratch, hipStream_t st) {
    if (n > SCAN_PAIR_MAX) {
        hipError_t e = exclusive_scan(a, n, oa, scratch, st);
        return e != hipSuccess ? e : exclusive_scan(b, n, ob, scratch, st);
    }
    hipLaunchKernelGGL(scan_pair_kernel, dim3(1), dim3(1024), 0, st, a, b, n, oa, ob);
    return hipGetLastError();
}

hipError_t exclusive_scan(const int64_t* in, int64_t n, int64_t* out, int64_t* scratch, hipStream_t st) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) return hipMemcpyAsync(out, scratch, 0, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nb), dim3(256), 0, st, in, n, scratch);
    hipLaunchKernelGGL(scan_block_offsets, dim3(1), dim3(1024), 0, st, scratch, nb);
    hipLaunchKernelGGL(scan_finish, dim3((unsigned)nb), dim3(256), 0, st, in, n, scratch, out);
    return hipGetLastError();
}

hipError_t launch_exact_count(const DGraph& g, const Plan& p, uint64_t nfirst, int group, int blocks, TicketPlan tp,
                              unsigned long long* ticket, unsigned long long* partials, unsigned long long* out2,
                              const uint32_t* elist, hipStream_t st) {
    PackedPlan pp{};
    for (int j = 0; j < 8; ++j) {
        pp.connect |= (uint64_t)p.connect[j] << (8 * j);
        pp.disconnect |= (uint64_t)p.disconnect[j] << (8 * j);
        pp.upper |= (uint64_t)p.upper[j] << (8 * j);
        pp.lower |= (uint64_t)p.lower[j] << (8 * j);
    }
    pp.k = p.k;
    pp.oriented = p.oriented;
    if (group == 8)
        hipLaunchKernelGGL(exact_count_kernel<8>, dim3((unsigned)blocks), dim3(256), 0, st, g, pp, nfirst, tp,
                           ticket, partials, elist);
    else if (group == 16)
        hipLaunchKernelGGL(exact_count_kernel<16>, dim3((unsigned)blocks), dim3(256), 0, st, g, pp, nfirst, tp,
                           ticket, partials, elist);
    else if (group == 64)
        hipLaunchKernelGGL(exact_count_kernel<64>, dim3((unsigned)blocks), dim3(256), 0, st, g, pp, nfirst, tp,
                           ticket, partials, elist);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(256), 0, st, partials, blocks, out2);
    return hipGetLastError();
}

hipError_t launch_clique_bitmap(const DGraph& g, int k, uint64_t nfirst, int blocks, TicketPlan tp,
                                unsigned long long* ticket, unsigned long long* partials, unsigned long long* out2,
                                uint32_t* overflow, unsigned long long* noverflow, hipStream_t st) {
    if (k == 4)
        hipLaunchKernelGGL(clique_bitmap_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, g, nfirst, tp,
                           ticket, partials, overflow, noverflow);
    else if (k == 5)
        hipLaunchKernelGGL(clique_bitmap_kernel<5>, dim3((unsigned)blocks), dim3(256), 0, st, g, nfirst, tp,
                           ticket, partials, overflow, noverflow);
    else if (k == 6)
        hipLaunchKernelGGL(clique_bitmap_kernel<6>, dim3((unsigned)blocks), dim3(256), 0, st, g, nfirst, tp,
                           ticket, partials, overflow, noverflow);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(256), 0, st, partials, blocks, out2);
    return hipGetLastError();
}

hipError_t launch_clique_bitmap128(const DGraph& g, int k, const uint32_t* elist, uint64_t nlist, int blocks,
                                   TicketPlan tp, unsigned long long* ticket, unsigned long long* partials,
                                   unsigned long long* out2, uint32_t* overflow, unsigned long long* noverflow,
                                   hipStream_t st) {
    if (k == 4)
        hipLaunchKernelGGL(clique_bitmap128_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, g, elist, nlist, tp,
                           ticket, partials, overflow, noverflow);
    else if (k == 5)
        hipLaunchKernelGGL(clique_bitmap128_kernel<5>, dim3((unsigned)blocks), dim3(256), 0, st, g, elist, nlist, tp,
                           ticket, partials, overflow, noverflow);
    else if (k == 6)
        hipLaunchKernelGGL(clique_bitmap128_kernel<6>, dim3((unsigned)blocks), dim3(256), 0, st, g, elist, nlist, tp,
                           ticket, partials, overflow, noverflow);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(256), 0, st, partials, blocks, out2);
    return hipGetLastError();
}

int clique_bitmap128_blocks_per_cu(int k) {
    int nb = 0;
    hipError_t e = k == 4   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, clique_bitmap128_kernel<4>, 256, 0)
                   : k == 5 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, clique_bitmap128_kernel<5>, 256, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, clique_bitmap128_kernel<6>, 256, 0);
    if (e != hipSuccess || nb < 1) nb = 2;
    return nb;
}

hipError_t launch_edge_terms(const DGraph& g, int group, bool need_t, int blocks, TicketPlan tp, const int sel[3],
                             unsigned long long* ticket, unsigned long long* partials, unsigned long long* out6,
                             hipStream_t st) {
    if (!need_t)
        hipLaunchKernelGGL((edge_terms_kernel<64, false>), dim3((unsigned)blocks), dim3(256), 0, st, g, tp, sel[0],
                           sel[1], sel[2], ticket, partials);
    else if (group == 8)
        hipLaunchKernelGGL((edge_terms_kernel<8, true>), dim3((unsigned)blocks), dim3(256), 0, st, g, tp, sel[0],
                           sel[1], sel[2], ticket, partials);
    else if (group == 64)
        hipLaunchKernelGGL((edge_terms_kernel<64, true>), dim3((unsigned)blocks), dim3(256), 0, st, g, tp, sel[0],
                           sel[1], sel[2], ticket, partials);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_six_kernel, dim3(1), dim3(256), 0, st, partials, blocks, out6);
    return hipGetLastError();
}

int edge_terms_blocks_per_cu(int group, bool need_t) {
    int nb = 0;
    hipError_t e = !need_t       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, edge_terms_kernel<64, false>, 256, 0)
                   : group == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, edge_terms_kernel<8, true>, 256, 0)
                                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, edge_terms_kernel<64, true>, 256, 0);
    if (e != hipSuccess || nb < 1) nb = 2;
    return nb;
}

// The allocation-free count's scratch.  In host code `scratch` names a host
// stand-in, not device memory: kernels and copies only ever get the address
// hipGetSymbolAddress returns for it on the current device, kept per device.
static __device__ __align__(256) unsigned long long scratch[kCountScratchWords];

hipError_t count_scratch_address(int dev, unsigned long long** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned long long* addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        addr[dev] = (unsigned long long*)ptr;
    }
    *out = addr[dev];
    return hipSuccess;
}

int clique_bitmap_blocks_per_cu(int k) {
    int nb = 0;
    hipError_t e = k == 4   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, clique_bitmap_kernel<4>, 256, 0)
                   : k == 5 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, clique_bitmap_kernel<5>, 256, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, clique_bitmap_kernel<6>, 256, 0);
    if (e != hipSuccess || nb < 1) nb = 2;
    return nb;
}

int exact_blocks_per_cu(int group) {
    int nb = 0;
    hipError_t e = group == 8    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, exact_count_kernel<8>, 256, 0)
                   : group == 16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, exact_count_kernel<16>, 256, 0)
                                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, exact_count_kernel<64>, 256, 0);
    if (e != hipSuccess || nb < 1) nb = 2;
    return nb;
}

}  // namespace sgpm
