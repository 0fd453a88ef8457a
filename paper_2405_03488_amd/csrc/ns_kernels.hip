// NS-prune sampling kernels for gfx950 (wave64).
//
// One launch processes the sample ids [s0, s1) of one convergence window
// (NS-online algorithm, Sec. 4.1).  Each sample (NS-prune, Sec. 4.2):
//   * draws its first edge uniformly: from the m oriented edges (v0 > v1) when
//     the plan orders them, else from the 2m arcs; alpha = m or 2m;
//   * for every later position j builds the candidate set S_j = members of the
//     smallest connected earlier row that lie inside the symmetry-breaking
//     bounds, are adjacent to every other connected earlier vertex, are not
//     adjacent to the disconnected ones (vertex-induced counting) and differ
//     from all earlier vertices; an empty S_j ends the sample as a miss;
//   * picks member floor(|S_j| * r / 2^64) of S_j in ascending order and
//     multiplies alpha by |S_j| (the inverse selection probability);
//   * on reaching the last position is a hit with X = alpha.
// Draw d of sample s is Philox4x32-10 (Salmon et al., SC'11) with key = seed
// and counter = (s lo, s hi, d, tag), read as w1*2^32 + w0.
//
// Work distribution: a wave takes tickets of (64 / G) * spl consecutive sample
// ids from NTK atomic counters (XCD-local first, then the others); G lanes cooperate on one sample (G = 1: one lane
// per sample with cursor-advancing binary searches; G > 1: the group scans the
// driver row G entries at a time, tests membership lane-parallel and counts
// with ballot + popcount).  Any G gives the same samples.
//
// Sums: each lane accumulates X into a 192-bit and X^2 into a 320-bit integer;
// the block turns them into 32-bit digits, adds, normalises and writes a
// 20-word partial; the launch's last block adds the partials.  Integer
// addition makes the result independent of the schedule.
#include "ns_device.h"

namespace sgpm {

// Sum of `nrows` 20-word rows (nrows <= 64) into out[0..PF_N) by the block:
// thread t < 240 adds column t % 20 of rows t / 20, t / 20 + 12, ... (at most
// six independent loads), then 20 threads add the 12 part sums.  `red` holds
// 240 words of LDS.
__device__ __forceinline__ void sum_rows(const unsigned long long* rows, int nrows, unsigned long long* out,
                                         unsigned long long* red) {
    const int t = (int)threadIdx.x;
    if (t < 240) {
        const int col = t % PF_N;
        unsigned long long a = 0;
        for (int r = t / PF_N; r < nrows; r += 240 / PF_N) a += rows[(size_t)r * PF_N + col];
        red[t] = a;
    }
    __syncthreads();
    if (t < PF_N) {
        unsigned long long a = 0;
        for (int k = 0; k < 240 / PF_N; ++k) a += red[k * PF_N + t];
        out[t] = a;
    }
    __syncthreads();
}

// End of a sampling launch, after this block's partial (20 words at
// partials[blockIdx.x]) is written: the partials are added in a two-level
// tree.  Blocks finish in groups of FIN_GROUP; the last block of a group to
// finish adds the group's partials into a group partial (after the launch's
// block partials), and the last group to finish adds the group partials into
// `out` (host-mapped, 20 words) and clears the ticket counters and the finish
// counts, so the next launch on this slot starts from zero.  Each finish count
// is taken after a release fence, and its last taker fences (acquire) before
// reading: the blocks run on different XCDs, whose L2s are not coherent.
// `ticket`: NTK counters TK_STRIDE words apart, then the counts FIN_STRIDE
// words apart (index 0: the groups, 1 + g: group g).  `red`: 240 words of LDS.
__device__ __forceinline__ void fold_launch(unsigned long long* partials, unsigned long long* ticket,
                                            unsigned long long* out, unsigned long long* red, int* flag) {
    unsigned long long* fin = ticket + (size_t)NTK * TK_STRIDE;
    const int nb = (int)gridDim.x, ng = (nb + FIN_GROUP - 1) / FIN_GROUP, gi = (int)blockIdx.x / FIN_GROUP;
    const int gsize = min(FIN_GROUP, nb - gi * FIN_GROUP);
    unsigned long long* gpart = partials + (size_t)nb * PF_N;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long old = atomicAdd(fin + (size_t)(1 + gi) * FIN_STRIDE, 1ull);
        *flag = old + 1ull == (unsigned long long)gsize ? 1 : 0;
    }
    __syncthreads();
    if (!*flag) return;
    __threadfence();
    sum_rows(partials + (size_t)gi * FIN_GROUP * PF_N, gsize, gpart + (size_t)gi * PF_N, red);
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long old = atomicAdd(fin, 1ull);
        *flag = old + 1ull == (unsigned long long)ng ? 1 : 0;
    }
    __syncthreads();
    if (!*flag) return;
    __threadfence();
    sum_rows(gpart, ng, out, red);
    const int t = (int)threadIdx.x;
    if (t < NTK) ticket[(size_t)t * TK_STRIDE] = 0ull;
    else if (t < NTK + 1 + ng) fin[(size_t)(t - NTK) * FIN_STRIDE] = 0ull;
    __threadfence_system();  // `out` is host memory read after the stream's next event
}

template <int G>
__global__ __launch_bounds__(256) void ns_window_kernel(DGraph g, Plan p, uint64_t seed, uint32_t tag, uint64_t s0,
                                                        uint64_t s1, int spl, unsigned long long* __restrict__ ticket,
                                                        unsigned long long* __restrict__ partials,
                                                        unsigned long long* __restrict__ out, int checksum,
                                                        int count_bytes, TraceArgs tr) {
    const int lane = (int)(threadIdx.x & 63);
    const bool leader = (lane & (G - 1)) == 0;
    const uint64_t per_wave = (uint64_t)(64 / G) * (uint64_t)spl;
    __shared__ __align__(16) int32_t s_list[LDS_WORDS];
    int32_t* list = s_list + (threadIdx.x / G) * (LDS_WORDS / (256 / G));
    Acc a;
#pragma unroll
    for (int i = 0; i < 3; ++i) a.s1[i] = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) a.s2[i] = 0;
    a.hits = a.csum = a.bytes = a.ovf = 0;

    const uint64_t ntickets = (s1 - s0 + per_wave - 1) / per_wave;
    int tk_cur = (int)(blockIdx.x % NTK), tk_left = NTK;
    for (;;) {
        uint64_t t = 0;
        if (!next_ticket(ticket, ntickets, tk_cur, tk_left, t)) break;
        const uint64_t base = s0 + t * per_wave;
        if (base >= s1) break;
        for (int q = 0; q < spl; ++q) {
            const uint64_t s = base + (uint64_t)q * (uint64_t)(64 / G) + (uint64_t)(lane / G);
            if (s >= s1) break;
            int32_t v[8];
            uint64_t alo, ahi, b = 0;
            const uint32_t st = ns_sample<G>(g, p, seed, tag, s, v, alo, ahi, a.ovf, b, count_bytes != 0, list);
            if (!leader) continue;
            if (st != 0xFFu) {
                alo = 0;
                ahi = 0;
            } else {
                a.hits += 1;
                acc_add(a, alo, ahi);
            }
            a.bytes += b;
            if (checksum) {
                uint64_t h = fmix64(s ^ 0x9E3779B97F4A7C15ull);
                h = fmix64(h ^ (uint64_t)st);
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (i < p.k) h = fmix64(h ^ (uint64_t)(uint32_t)v[i]);
                h = fmix64(h ^ alo);
                h = fmix64(h ^ ahi);
                a.csum += h;
            }
            if (tr.buf && s >= tr.lo && s < tr.hi) {
                sgpm_trace_rec* r = tr.buf + (s - tr.lo);
                r->s = s;
#pragma unroll
                for (int i = 0; i < 8; ++i) r->v[i] = v[i];
                r->status = st;
                r->k = (uint32_t)p.k;
                r->alpha_lo = alo;
                r->alpha_hi = ahi;
            }
        }
    }

    // block reduction into 32-bit digits
    unsigned long long f[PF_N];
    f[0] = a.s1[0] & 0xFFFFFFFFull;
    f[1] = a.s1[0] >> 32;
    f[2] = a.s1[1] & 0xFFFFFFFFull;
    f[3] = a.s1[1] >> 32;
    f[4] = a.s1[2] & 0xFFFFFFFFull;
    f[5] = a.s1[2] >> 32;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        f[6 + 2 * i] = a.s2[i] & 0xFFFFFFFFull;
        f[7 + 2 * i] = a.s2[i] >> 32;
    }
    f[PF_HITS] = a.hits;
    f[PF_CSUM] = a.csum;
    f[PF_BYTES] = a.bytes;
    f[PF_OVF] = a.ovf;
    __shared__ unsigned long long red[4][PF_N];
    const int w = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int i = 0; i < PF_N; ++i) {
        const unsigned long long x = wave_sum(f[i]);
        if (lane == 0) red[w][i] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long o[PF_N];
#pragma unroll
        for (int i = 0; i < PF_N; ++i) o[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
        // normalise digit blocks (S1: 6 digits, S2: 10 digits)
        // (the top digit of each block keeps any excess; the host adds digits
        // with full carries)
        unsigned long long c = 0;
        for (int i = 0; i < 5; ++i) {
            const unsigned long long t = o[i] + c;
            o[i] = t & 0xFFFFFFFFull;
            c = t >> 32;
        }
        o[5] += c;
        c = 0;
        for (int i = 6; i < 15; ++i) {
            const unsigned long long t = o[i] + c;
            o[i] = t & 0xFFFFFFFFull;
            c = t >> 32;
        }
        o[15] += c;
        unsigned long long* dst = partials + (size_t)blockIdx.x * PF_N;
        for (int i = 0; i < PF_N; ++i) dst[i] = o[i];
    }
    __shared__ int s_last;
    fold_launch(partials, ticket, out, reinterpret_cast<unsigned long long*>(s_list), &s_last);
}

// One sample per wave, samples handled in groups of up to GMAX per wave:
//  * prologue: the group's Philox draws are evaluated at once, one (sample,
//    draw) pair per lane; a sample reads its draws back with readlane;
//  * each sample leaves a record (walk, status, weight, bytes) in LDS;
//  * epilogue: lane q hashes record q and forms the 32-bit digits of its
//    weight and the digit columns of the weight's square, and adds them to the
//    wave's sums in LDS (LDS atomics); the sums are normalised once per block.
// MODE 0: uniform proposal; 1: learned proposal; 2: uniform with per-step set
// sizes recorded for traced samples (training pilots); 3: the NS-base sampler
// (lazy verification), which the paper measures NS-prune against.  CLQ: the plan is the
// K-clique's, so every plan test folds at compile time; this build also leaves
// out the trace and byte-count code, which halves the per-sample loop's
// uniform-register spills to vector lanes.
// Blocks per CU each one-sample-per-wave kernel is compiled for: the uniform
// clique kernels fit 64 VGPRs with their per-sample loop free of spills, and
// eight blocks keep 8 % more samples in flight; the others need 72 VGPRs.
constexpr int wave_occupancy(int mode, bool clq) { return clq && mode == 0 ? 8 : 7; }
constexpr int GMAX = 16;  // samples per group (records live in lanes 0..15)
constexpr int REC = 16;   // words per sample record

// draw index held in slot t of a sample's draws (slots 0..k-2: draws 0, 2, ..,
// k-1; learned proposal: then draws 18, .., 16 + k-2 of its weighted steps)
template <int K>
__device__ __forceinline__ uint32_t draw_of_slot(int t) {
    return t == 0 ? 0u : t <= K - 2 ? (uint32_t)(t + 1) : (uint32_t)(18 + (t - (K - 1)));
}

template <int MODE, int K, bool CLQ>
__global__ __launch_bounds__(256, wave_occupancy(MODE, CLQ)) void ns_wave_kernel(DGraph g, Plan p, uint64_t seed, uint32_t tag, uint64_t s0,
                                                      uint64_t s1, int spl, unsigned long long* __restrict__ ticket,
                                                      unsigned long long* __restrict__ partials,
                                                      unsigned long long* __restrict__ out, int checksum,
                                                      int count_bytes, TraceArgs tr, LearnArgs la) {
    constexpr int G = 64;
    constexpr int D = (K - 1) + (MODE == 1 && K > 3 ? K - 3 : 0);  // draws per sample
    constexpr int GS = (64 / D) < GMAX ? (64 / D) : GMAX;
    const int lane = (int)(threadIdx.x & 63);
    const int wid = (int)(threadIdx.x >> 6);
    __shared__ __align__(16) int32_t s_list[LDS_WORDS];
    __shared__ uint32_t s_hist[4][32];
    __shared__ __align__(16) uint32_t s_rec[4][GMAX * REC];
    __shared__ unsigned long long s_wsum[4][16];
    uint32_t* hist = s_hist[wid];
    uint32_t* rec = s_rec[wid];
    unsigned long long* wsum = s_wsum[wid];
    int32_t* list = s_list + wid * (LDS_WORDS / 4);
    if (lane < 16) wsum[lane] = 0ull;
    // the learned proposal's bucket thresholds, one per lane, held for the launch
    LearnArgs lal = la;
    lal.lane_thr = (MODE == 1 && la.thr && lane < 32) ? la.thr[lane] : 0;
    __builtin_amdgcn_wave_barrier();
    uint64_t ovf = 0;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t tstat = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t ntickets = (s1 - s0 + (uint64_t)spl - 1) / (uint64_t)spl;
    int tk_cur = (int)(blockIdx.x % NTK), tk_left = NTK;
    // tickets 0 .. nwaves-1 go to the waves by index, without an atomic (the
    // launch's first fetches would all hit the counters at once); the rest
    // come from the counters
    bool first = true;
    const uint64_t ndyn = ntickets > nwaves ? ntickets - nwaves : 0;
    for (;;) {
        uint64_t tt = 0;
        if (first) {
            first = false;
            tt = tstat;
        } else {
            uint64_t td = 0;
            if (ndyn == 0 || !next_ticket(ticket, ndyn, tk_cur, tk_left, td)) break;
            tt = nwaves + td;
        }
        const uint64_t base = s0 + tt * (uint64_t)spl;
        if (base >= s1) break;
        const uint64_t end = min(s1, base + (uint64_t)spl);
        for (uint64_t gb = base; gb < end; gb += (uint64_t)GS) {
            const int n = (int)min((uint64_t)GS, end - gb);
            // prologue: every draw of the group, lane (q * D + t) holding draw slot t of sample gb + q
            Draws dr;
            {
                const int q = lane / D, t = lane - q * D;
                uint64_t r = 0;
                if (q < n) r = philox_r64(seed, gb + (uint64_t)q, draw_of_slot<K>(t), tag);
                dr.lo = (uint32_t)r;
                dr.hi = (uint32_t)(r >> 32);
                dr.k1 = K - 1;
                dr.base = 0;
            }
            // heads: every sample's first edge and row bounds, loaded at once
            if constexpr (MODE != 3) prefetch_heads(g, CLQ || p.oriented, dr, D, n, rec, REC, MODE == 1 ? &lal : nullptr);
            for (int q = 0; q < n; ++q) {
                const uint64_t s = gb + (uint64_t)q;
                dr.base = q * D;
                Head hd;
                if constexpr (MODE != 3) hd = read_head(rec + q * REC, MODE == 1);
                int32_t v[8];
                uint64_t alo, ahi, b = 0, ov = 0;
                uint32_t sz[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                uint32_t st;
                if constexpr (MODE == 3)
                    st = ns_base_sample<K>(g, p, seed, tag, s, v, alo, ahi, ov, list, &dr);
                else
                    st = ns_sample<G, K, CLQ>(g, p, seed, tag, s, v, alo, ahi, ov, b, !CLQ && count_bytes != 0, list,
                                              MODE == 1 ? &lal : nullptr, hist, MODE == 2 ? sz : nullptr, &dr, &hd);
                ovf |= ov;
                if (st != 0xFFu) {
                    alo = 0;
                    ahi = 0;
                }
                // the sample's record (words 0-7 the walk, 8 the status, 9-12 X,
                // 13-14 bytes), written by lane 0 from the uniform registers
                if (lane == 0) write_record<K>(rec + q * REC, v, st, alo, ahi, b);
                if (!CLQ && tr.buf && s >= tr.lo && s < tr.hi && lane < 16) {
                    uint32_t w = 0;
                    if (lane < 2) {
                        w = (uint32_t)(s >> (32 * lane));
                    } else if (lane < 10) {
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (lane - 2 == i) w = (uint32_t)v[i];
                    } else if (lane == 10) w = st;
                    else if (lane == 11) w = (uint32_t)p.k;
                    else if (lane < 14) w = (uint32_t)(alo >> (32 * (lane - 12)));
                    else w = (uint32_t)(ahi >> (32 * (lane - 14)));
                    reinterpret_cast<uint32_t*>(tr.buf + (s - tr.lo))[lane] = w;
                    if (MODE == 2 && tr.sizes && lane < 8) {
                        uint32_t z = 0;
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (lane == i) z = sz[i];
                        tr.sizes[(s - tr.lo) * 8 + (uint64_t)lane] = z;
                    }
                }
            }
            // epilogue: lane q < n takes sample gb + q (LDS operations of a wave
            // complete in order) and adds its columns to the wave's LDS sums
            __builtin_amdgcn_wave_barrier();
            if (lane < n) {
                const uint32_t* r = rec + lane * REC;
                const uint32_t st = r[8];
                uint32_t d[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) d[i] = r[9 + i];
                if (checksum) {
                    uint64_t h = fmix64((gb + (uint64_t)lane) ^ 0x9E3779B97F4A7C15ull);
                    h = fmix64(h ^ (uint64_t)st);
#pragma unroll
                    for (int i = 0; i < K; ++i) h = fmix64(h ^ (uint64_t)r[i]);
                    h = fmix64(h ^ ((uint64_t)d[1] << 32 | d[0]));
                    h = fmix64(h ^ ((uint64_t)d[3] << 32 | d[2]));
                    atomicAdd(&wsum[12], (unsigned long long)h);
                }
                if (!CLQ && count_bytes) atomicAdd(&wsum[13], (unsigned long long)((uint64_t)r[14] << 32 | r[13]));
                if (st == 0xFFu) {
                    // digits of X and the digit columns of X^2 (low and high halves of the digit products)
                    uint64_t c2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint64_t pr = (uint64_t)d[a] * (uint64_t)d[e];
                            c2[a + e] += pr & 0xFFFFFFFFull;
                            if (a + e + 1 < 8) c2[a + e + 1] += pr >> 32;
                        }
#pragma unroll
                    for (int i = 0; i < 4; ++i) atomicAdd(&wsum[i], (unsigned long long)d[i]);
#pragma unroll
                    for (int i = 0; i < 8; ++i) atomicAdd(&wsum[4 + i], (unsigned long long)c2[i]);
                    atomicAdd(&wsum[14], 1ull);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    __builtin_amdgcn_wave_barrier();
    // per wave: lanes 0-3 the digit sums of S1, 4-11 the column sums of S2,
    // 12 checksum, 13 bytes, 14 hits, 15 the overflow flag
    uint64_t acc = lane < 15 ? (uint64_t)wsum[lane] : 0ull;
    if (lane == 15) acc = ovf;
    // block reduction of the waves' sums
    __shared__ unsigned long long red[4][16];
    if (lane < 16) red[wid][lane] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long col[16];
        for (int i = 0; i < 16; ++i) col[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
        unsigned long long o[PF_N];
        for (int i = 0; i < PF_N; ++i) o[i] = 0;
        unsigned long long c = 0;
        for (int i = 0; i < 6; ++i) {  // S1: digit sums 0-3, carried into 6 digits
            const unsigned long long t = (i < 4 ? col[i] : 0ull) + c;
            o[PF_S1 + i] = i < 5 ? (t & 0xFFFFFFFFull) : t;
            c = t >> 32;
        }
        c = 0;
        for (int i = 0; i < 10; ++i) {  // S2: digit columns 0-7, carried into 10 digits
            const unsigned long long t = (i < 8 ? col[4 + i] : 0ull) + c;
            o[PF_S2 + i] = i < 9 ? (t & 0xFFFFFFFFull) : t;
            c = t >> 32;
        }
        o[PF_HITS] = col[14];
        o[PF_CSUM] = col[12];
        o[PF_BYTES] = col[13];
        o[PF_OVF] = col[15];
        unsigned long long* dst = partials + (size_t)blockIdx.x * PF_N;
        for (int i = 0; i < PF_N; ++i) dst[i] = o[i];
    }
    __shared__ int s_last;
    fold_launch(partials, ticket, out, reinterpret_cast<unsigned long long*>(s_list), &s_last);
}

__global__ void fill_u64_kernel(unsigned long long* p, uint64_t n, unsigned long long v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// one-sample-per-wave kernels, specialised on the pattern size so only the
// steps a pattern has are compiled into its kernel

// the plan is the k-clique's: every earlier position connected and above the
// new one, no disconnect or lower bounds, S_j inside S_{j-1} from j = 3
bool plan_is_clique(const Plan& p) {
    if (!p.oriented || p.k < 3) return false;
    for (int j = 1; j < p.k; ++j) {
        const uint32_t all = (1u << j) - 1u;
        if (p.connect[j] != all || p.upper[j] != all || p.disconnect[j] != 0 || p.lower[j] != 0) return false;
        if (j >= 3 && !p.reuse[j]) return false;
    }
    return true;
}

// whether a one-sample-per-wave launch takes the clique specialisation: a
// clique plan, no trace or byte count (the generic kernel computes the same
// walks and serves those requests), not the pilots' set-size mode
bool wave_uses_clique_kernel(const Plan& p, const TraceArgs& tr, const LearnArgs& la, int count_bytes) {
    return plan_is_clique(p) && p.k <= 6 && !tr.buf && !count_bytes && (la.table || !tr.sizes);
}

template <int MODE>
hipError_t launch_wave_mode(const DGraph& g, const Plan& p, uint64_t seed, uint32_t tag, uint64_t s0, uint64_t s1,
                            const LaunchCfg& cfg, unsigned long long* ticket, unsigned long long* partials, unsigned long long* out,
                            int checksum, int count_bytes, const TraceArgs& tr, const LearnArgs& la, hipStream_t st) {
    const dim3 grid((unsigned)cfg.blocks), block(256);
    const bool clq = MODE < 2 && wave_uses_clique_kernel(p, tr, la, count_bytes);
#define SGPM_WAVE_CASE(KK)                                                                                        \
    case KK:                                                                                                      \
        if (MODE < 2 && clq && KK >= 3 && KK <= 6)                                                                \
            hipLaunchKernelGGL((ns_wave_kernel<MODE, KK, MODE < 2 && KK >= 3 && KK <= 6>), grid, block, 0, st, g, p, \
                               seed, tag, s0, s1, cfg.spl, ticket, partials, out, checksum, count_bytes, tr, la); \
        else                                                                                                      \
            hipLaunchKernelGGL((ns_wave_kernel<MODE, KK, false>), grid, block, 0, st, g, p, seed, tag, s0, s1,    \
                               cfg.spl, ticket, partials, out, checksum, count_bytes, tr, la);                    \
        break;
    switch (p.k) {
        SGPM_WAVE_CASE(2)
        SGPM_WAVE_CASE(3)
        SGPM_WAVE_CASE(4)
        SGPM_WAVE_CASE(5)
        SGPM_WAVE_CASE(6)
        SGPM_WAVE_CASE(7)
        SGPM_WAVE_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef SGPM_WAVE_CASE
    return hipGetLastError();
}

hipError_t launch_wave(const DGraph& g, const Plan& p, uint64_t seed, uint32_t tag, uint64_t s0, uint64_t s1,
                       const LaunchCfg& cfg, unsigned long long* ticket, unsigned long long* partials, unsigned long long* out, int checksum,
                       int count_bytes, const TraceArgs& tr, const LearnArgs& la, hipStream_t st) {
    if (cfg.base) return launch_wave_mode<3>(g, p, seed, tag, s0, s1, cfg, ticket, partials, out, checksum, 0, tr, la, st);
    if (la.table) return launch_wave_mode<1>(g, p, seed, tag, s0, s1, cfg, ticket, partials, out, checksum, count_bytes, tr, la, st);
    if (tr.sizes) return launch_wave_mode<2>(g, p, seed, tag, s0, s1, cfg, ticket, partials, out, checksum, count_bytes, tr, la, st);
    return launch_wave_mode<0>(g, p, seed, tag, s0, s1, cfg, ticket, partials, out, checksum, count_bytes, tr, la, st);
}

hipError_t launch_ns_window(const DGraph& g, const Plan& p, uint64_t seed, uint32_t tag, uint64_t s0, uint64_t s1,
                            const LaunchCfg& cfg, unsigned long long* ticket, unsigned long long* partials, unsigned long long* out,
                            int checksum, int count_bytes, const TraceArgs& tr, const LearnArgs& la,
                            hipStream_t st) {
    const dim3 grid((unsigned)cfg.blocks), block(256);
    if ((la.table || tr.sizes || cfg.base) && cfg.lanes != 64) return hipErrorInvalidValue;
    switch (cfg.lanes) {
        case 1:
            hipLaunchKernelGGL(ns_window_kernel<1>, grid, block, 0, st, g, p, seed, tag, s0, s1, cfg.spl, ticket,
                               partials, out, checksum, count_bytes, tr);
            break;
        case 4:
            hipLaunchKernelGGL(ns_window_kernel<4>, grid, block, 0, st, g, p, seed, tag, s0, s1, cfg.spl, ticket,
                               partials, out, checksum, count_bytes, tr);
            break;
        case 16:
            hipLaunchKernelGGL(ns_window_kernel<16>, grid, block, 0, st, g, p, seed, tag, s0, s1, cfg.spl, ticket,
                               partials, out, checksum, count_bytes, tr);
            break;
        case 64:
            return launch_wave(g, p, seed, tag, s0, s1, cfg, ticket, partials, out, checksum, count_bytes, tr, la, st);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Resident 256-thread blocks per CU of the uniform clique kernels.
int ns_clique_blocks_per_cu() {
    static int cache = 0;
    if (cache) return cache;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ns_wave_kernel<0, 4, true>, 256, 0) != hipSuccess || nb < 1)
        nb = 1;
    cache = nb;
    return nb;
}

// Resident 256-thread blocks per CU for the sampling kernel of a lane count.
int ns_blocks_per_cu(int lanes) {
    static int cache[65] = {0};
    if (lanes < 1 || lanes > 64) return 1;
    if (cache[lanes]) return cache[lanes];
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (lanes) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ns_window_kernel<1>, 256, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ns_window_kernel<4>, 256, 0); break;
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ns_window_kernel<16>, 256, 0); break;
        case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ns_wave_kernel<0, 8, false>, 256, 0); break;
        default: break;
    }
    if (e != hipSuccess || nb < 1) nb = 2;
    cache[lanes] = nb;
    return nb;
}


}  // namespace sgpm
