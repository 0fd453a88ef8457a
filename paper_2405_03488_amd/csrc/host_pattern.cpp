// Pattern compiler: matching order + symmetry-breaking restrictions (Sec. 4.2).
//
// NS-prune stays unbiased as long as pruning keeps the one-to-one map between
// matches and root-to-leaf paths of the subgraph tree; matching order and
// symmetry breaking both do.  Rules (the paper cites GraphZero / G2Miner for
// them without fixing an algorithm):
//   order: the pattern vertex of largest degree (lowest id on ties), then its
//     largest-degree neighbour (lowest id on ties), then repeatedly the vertex
//     with the most edges into the matched prefix (ties: larger degree, lower
//     id);
//   restrictions: walk the positions in order; while the automorphisms that
//     fix all earlier positions still move position i, demand v_i > v_t for
//     each other position t of i's orbit, then keep only automorphisms fixing i
//     (orbit/stabiliser chain).  Every restriction ends up on its later
//     position t as "v_t < v_i" (bit i of upper[t]).
// The 4-cycle gives v0 > v1, v2, v3 and v1 > v3 as in the paper's example.
#include <algorithm>
#include <array>
#include <numeric>

#include "sgpm_internal.h"

namespace sgpm {

int compile_pattern(int k, int l, const int32_t* edges, int induced, Plan& out, std::string& err) {
    out = Plan{};
    if (k < 2 || k > 8) {
        err = "pattern must have 2..8 vertices";
        return SGPM_EUNSUPPORTED;
    }
    if (l < 0 || (l > 0 && !edges)) {
        err = "bad edge list";
        return SGPM_EINVAL;
    }
    std::array<uint32_t, 8> nb{};  // neighbour bitmask per pattern vertex
    for (int e = 0; e < l; e++) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b) {
            err = "pattern edge endpoint out of range or a loop";
            return SGPM_EINVAL;
        }
        nb[a] |= 1u << b;
        nb[b] |= 1u << a;
    }
    // connectivity by bitmask flood
    uint32_t reach = 1, prev = 0;
    while (reach != prev) {
        prev = reach;
        for (int a = 0; a < k; a++)
            if (reach >> a & 1) reach |= nb[a];
    }
    if (reach != (1u << k) - 1) {
        err = "pattern is disconnected";
        return SGPM_EUNSUPPORTED;
    }
    auto deg = [&](int a) { return __builtin_popcount(nb[a]); };
    // matching order
    std::array<int, 8> ord{};
    uint32_t placed = 0;
    int v0 = 0;
    for (int a = 0; a < k; a++)
        if (deg(a) > deg(v0)) v0 = a;
    int v1 = -1;
    for (int a = 0; a < k; a++)
        if ((nb[v0] >> a & 1) && (v1 < 0 || deg(a) > deg(v1))) v1 = a;
    ord[0] = v0;
    ord[1] = v1;
    placed = (1u << v0) | (1u << v1);
    for (int pos = 2; pos < k; pos++) {
        int pick = -1, links = -1;
        for (int a = 0; a < k; a++) {
            if (placed >> a & 1) continue;
            int c = __builtin_popcount(nb[a] & placed);
            if (c > links || (c == links && deg(a) > deg(pick))) {
                pick = a;
                links = c;
            }
        }
        ord[pos] = pick;
        placed |= 1u << pick;
    }
    // automorphisms mapped onto positions
    std::array<int, 8> where{};
    for (int i = 0; i < k; i++) where[ord[i]] = i;
    std::vector<std::array<int8_t, 8>> auts;
    std::array<int, 8> pi{};
    std::iota(pi.begin(), pi.begin() + k, 0);
    do {
        bool ok = true;
        for (int a = 0; a < k && ok; a++) {
            uint32_t img = 0;
            for (int b = 0; b < k; b++)
                if (nb[a] >> b & 1) img |= 1u << pi[b];
            ok = img == nb[pi[a]];
        }
        if (ok) {
            std::array<int8_t, 8> g{};
            for (int i = 0; i < k; i++) g[i] = (int8_t)where[pi[ord[i]]];
            auts.push_back(g);
        }
    } while (std::next_permutation(pi.begin(), pi.begin() + k));
    out.aut = (int32_t)auts.size();
    // orbit / stabiliser chain
    std::vector<std::array<int8_t, 8>> stab = auts;
    for (int i = 0; i < k; i++) {
        uint32_t orbit = 0;
        for (auto& g : stab) orbit |= 1u << g[i];
        orbit &= ~(1u << i);
        for (int t = i + 1; t < k; t++)
            if (orbit >> t & 1) out.upper[t] |= (uint8_t)(1u << i);
        std::vector<std::array<int8_t, 8>> keep;
        for (auto& g : stab)
            if (g[i] == i) keep.push_back(g);
        stab.swap(keep);
    }
    out.k = k;
    out.induced = induced ? 1 : 0;
    for (int i = 0; i < k; i++) out.order[i] = ord[i];
    for (int j = 1; j < k; j++)
        for (int i = 0; i < j; i++) {
            bool e = nb[ord[j]] >> ord[i] & 1;
            if (e) out.connect[j] |= (uint8_t)(1u << i);
            else if (induced) out.disconnect[j] |= (uint8_t)(1u << i);
        }
    out.oriented = (out.upper[1] & 1) ? 1 : 0;
    // steps whose constraint set contains the previous step's can filter the
    // previous candidate set instead of scanning a row again
    for (int j = 3; j < k; j++) {
        auto sub = [](uint8_t a, uint8_t b) { return (a & ~b) == 0; };
        out.reuse[j] = sub(out.connect[j - 1], out.connect[j]) && sub(out.disconnect[j - 1], out.disconnect[j]) &&
                       sub(out.upper[j - 1], out.upper[j]) && sub(out.lower[j - 1], out.lower[j]);
    }
    return SGPM_OK;
}

}  // namespace sgpm
