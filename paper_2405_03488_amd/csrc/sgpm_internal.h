// Internal types shared by the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/sgpm.h"

namespace sgpm {

// Compiled pattern (NS-prune plan, Sec. 4.2); passed to kernels by value.
struct Plan {
    int32_t k, oriented, induced, aut;
    int32_t order[8];
    uint8_t connect[8], disconnect[8], upper[8], lower[8];
};

// Device-resident canonical graph.
struct DGraph {
    const int64_t* off;   // [n+1]
    const int32_t* nbr;   // [2m] rows ascending
    const int2* epair;    // [m] oriented edges (u, w), w < u, in (u, w) order
    const int32_t* arow;  // [2m] row of each arc
    int64_t n, m;
};

// Per-block partial record written by the sampling kernels.
enum {
    PF_S1 = 0,    // 6 normalised 32-bit digits of sum X
    PF_S2 = 6,    // 10 normalised 32-bit digits of sum X^2
    PF_HITS = 16,
    PF_CSUM = 17,
    PF_BYTES = 18,
    PF_OVF = 19,
    PF_N = 20
};

struct TraceArgs {
    sgpm_trace_rec* buf;  // device buffer
    uint64_t lo, hi;
};

struct LaunchCfg {
    int lanes;     // lanes cooperating on one sample: 1, 4, 16, 64
    int spl;       // samples per group per ticket
    int blocks;    // grid size
};

// kernels (ns_kernels.hip)
hipError_t launch_ns_window(const DGraph& g, const Plan& p, uint64_t seed, uint32_t tag, uint64_t s0, uint64_t s1,
                            const LaunchCfg& cfg, unsigned long long* ticket, unsigned long long* partials,
                            int checksum, int count_bytes, const TraceArgs& tr, hipStream_t st);
hipError_t launch_reduce_partials(const unsigned long long* partials, int nblocks, unsigned long long* out20,
                                  hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t st);

// host helpers
struct HostGraph {
    int64_t n = 0, m = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> nbr;
    std::vector<int32_t> perm;  // perm[original] = canonical
};
int canonicalise(int64_t n, const void* offsets, int off64, const int32_t* nbrs, bool assume_canonical,
                 HostGraph& out, std::string& err);
int compile_pattern(int k, int l, const int32_t* edges, int induced, Plan& out, std::string& err);

// exact big integers as little-endian 32-bit digits
struct Big {
    std::vector<uint32_t> d;
    explicit Big(size_t nd = 24) : d(nd, 0) {}
};
void big_add_digits(Big& a, const unsigned long long* digits, int nd);  // digits may exceed 32 bits
double big_to_double(const Big& a);
bool big_is_zero(const Big& a);
double normal_quantile(double p);
double predicted_error(double z, uint64_t n, const Big& S1, const Big& S2);
uint64_t next_window_end(uint64_t n_t, const sgpm_options& o);

}  // namespace sgpm
