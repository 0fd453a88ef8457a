// Graph loader: canonical CSR with degree-ordered relabelling.
//
// The paper keeps its data graphs symmetric with no loops or duplicate edges,
// stored as CSR, and orients them for cliques (Sec. 6 and its data-graph
// table).  Canonical form here: symmetrise, drop loops and duplicates, relabel
// vertices by degree descending (ties: original id ascending) and sort every
// row ascending.  With that relabelling a restriction "v_j < v_i" points the
// walk at higher-degree vertices and the prefix of each row below a bound is
// its oriented (lower) neighbourhood.
//
// Host implementation: multithreaded bucket scatter with atomic row cursors,
// per-row sort/unique, then a counting sort by degree for the relabel.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>

#include "sgpm_internal.h"

namespace sgpm {

static int num_threads() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 1;
    return (int)std::min(h, 16u);
}

// Dynamic parallel for over [0, n) in chunks.
template <class F>
static void parallel_for(int64_t n, int64_t chunk, F f) {
    int nt = num_threads();
    if (n <= chunk || nt == 1) {
        for (int64_t i = 0; i < n; i++) f(i);
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    for (int t = 0; t < nt; t++)
        th.emplace_back([&]() {
            for (;;) {
                int64_t b = next.fetch_add(chunk);
                if (b >= n) break;
                int64_t e = std::min(n, b + chunk);
                for (int64_t i = b; i < e; i++) f(i);
            }
        });
    for (auto& x : th) x.join();
}

static bool read_offsets(int64_t n, const void* offsets, int off64, std::vector<int64_t>& o) {
    o.resize((size_t)n + 1);
    if (off64) std::memcpy(o.data(), offsets, sizeof(int64_t) * (size_t)(n + 1));
    else {
        const int32_t* p = (const int32_t*)offsets;
        for (int64_t i = 0; i <= n; i++) o[(size_t)i] = p[i];
    }
    if (o[0] != 0) return false;
    for (int64_t i = 0; i < n; i++)
        if (o[(size_t)i + 1] < o[(size_t)i]) return false;
    return true;
}

static bool is_canonical(int64_t n, const std::vector<int64_t>& off, const int32_t* nbr) {
    std::atomic<bool> ok(true);
    parallel_for(n, 4096, [&](int64_t u) {
        int64_t b = off[(size_t)u], e = off[(size_t)u + 1];
        if (u + 1 < n && e - b < off[(size_t)u + 2] - e) ok = false;  // degree descending
        for (int64_t i = b; i < e; i++) {
            int32_t v = nbr[i];
            if (v == u || (i > b && nbr[i - 1] >= v)) { ok = false; return; }
            // symmetric: u must be in row v
            const int32_t* rb = nbr + off[(size_t)v];
            const int32_t* re = nbr + off[(size_t)v + 1];
            const int32_t* f = std::lower_bound(rb, re, (int32_t)u);
            if (f == re || *f != u) { ok = false; return; }
        }
    });
    return ok;
}

int canonicalise(int64_t n, const void* offsets, int off64, const int32_t* nbrs, bool assume_canonical,
                 HostGraph& out, std::string& err) {
    std::vector<int64_t> in_off;
    if (!read_offsets(n, offsets, off64, in_off)) {
        err = "offsets are not a monotone CSR offset array starting at 0";
        return SGPM_EBADGRAPH;
    }
    const int64_t nin = in_off[(size_t)n];
    std::atomic<bool> bad(false);
    parallel_for(nin, 1 << 16, [&](int64_t i) {
        if (nbrs[i] < 0 || nbrs[i] >= n) bad = true;
    });
    if (bad) {
        err = "neighbour id out of range";
        return SGPM_EBADGRAPH;
    }
    out.n = n;
    if (assume_canonical) {
        if (!is_canonical(n, in_off, nbrs)) {
            err = "input is not canonical (symmetric, loop-free, sorted rows, degree descending)";
            return SGPM_EBADGRAPH;
        }
        out.off = in_off;
        out.nbr.assign(nbrs, nbrs + nin);
        out.perm.resize((size_t)n);
        for (int64_t i = 0; i < n; i++) out.perm[(size_t)i] = (int32_t)i;
        out.m = nin / 2;
        return SGPM_OK;
    }
    // 1. symmetric arc counts (with duplicates) per row
    std::vector<std::atomic<int64_t>> cur((size_t)n + 1);
    for (auto& c : cur) c.store(0, std::memory_order_relaxed);
    parallel_for(n, 1024, [&](int64_t u) {
        for (int64_t i = in_off[(size_t)u]; i < in_off[(size_t)u + 1]; i++) {
            int32_t v = nbrs[i];
            if (v == u) continue;
            cur[(size_t)u].fetch_add(1, std::memory_order_relaxed);
            cur[(size_t)v].fetch_add(1, std::memory_order_relaxed);
        }
    });
    std::vector<int64_t> roff((size_t)n + 1, 0);
    for (int64_t u = 0; u < n; u++) roff[(size_t)u + 1] = roff[(size_t)u] + cur[(size_t)u].load();
    for (int64_t u = 0; u < n; u++) cur[(size_t)u].store(roff[(size_t)u], std::memory_order_relaxed);
    std::vector<int32_t> raw((size_t)roff[(size_t)n]);
    // 2. scatter both directions
    parallel_for(n, 1024, [&](int64_t u) {
        for (int64_t i = in_off[(size_t)u]; i < in_off[(size_t)u + 1]; i++) {
            int32_t v = nbrs[i];
            if (v == u) continue;
            raw[(size_t)cur[(size_t)u].fetch_add(1, std::memory_order_relaxed)] = v;
            raw[(size_t)cur[(size_t)v].fetch_add(1, std::memory_order_relaxed)] = (int32_t)u;
        }
    });
    // 3. sort + unique each row; deg = distinct neighbours
    std::vector<int64_t> deg((size_t)n);
    parallel_for(n, 256, [&](int64_t u) {
        int32_t* b = raw.data() + roff[(size_t)u];
        int32_t* e = raw.data() + roff[(size_t)u + 1];
        std::sort(b, e);
        deg[(size_t)u] = std::unique(b, e) - b;
    });
    // 4. relabel: counting sort by degree descending, ids ascending within a degree
    int64_t maxdeg = 0;
    for (int64_t u = 0; u < n; u++) maxdeg = std::max(maxdeg, deg[(size_t)u]);
    std::vector<int64_t> start((size_t)maxdeg + 2, 0);
    for (int64_t u = 0; u < n; u++) start[(size_t)(maxdeg - deg[(size_t)u]) + 1]++;
    for (int64_t d = 0; d <= maxdeg; d++) start[(size_t)d + 1] += start[(size_t)d];
    out.perm.assign((size_t)n, 0);
    std::vector<int32_t> inv((size_t)n);
    for (int64_t u = 0; u < n; u++) {
        int64_t r = start[(size_t)(maxdeg - deg[(size_t)u])]++;
        out.perm[(size_t)u] = (int32_t)r;
        inv[(size_t)r] = (int32_t)u;
    }
    // 5. canonical rows
    out.off.assign((size_t)n + 1, 0);
    for (int64_t r = 0; r < n; r++) out.off[(size_t)r + 1] = out.off[(size_t)r] + deg[(size_t)inv[(size_t)r]];
    out.nbr.resize((size_t)out.off[(size_t)n]);
    parallel_for(n, 256, [&](int64_t r) {
        int32_t u = inv[(size_t)r];
        const int32_t* src = raw.data() + roff[(size_t)u];
        int32_t* dst = out.nbr.data() + out.off[(size_t)r];
        int64_t d = deg[(size_t)u];
        for (int64_t i = 0; i < d; i++) dst[i] = out.perm[(size_t)src[i]];
        std::sort(dst, dst + d);
    });
    out.m = out.off[(size_t)n] / 2;
    return SGPM_OK;
}

}  // namespace sgpm
