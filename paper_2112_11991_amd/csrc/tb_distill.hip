// tb_distill.hip -- candidate grouping on the host (App. A: repeated
// detections of one signal are grouped and the strongest one kept).
//
// A candidate's fundamental sits at F = 16 k / h = k << (4 - log2_harm)
// sixteenths of a fundamental bin.  Candidates are taken from the strongest
// (sigma descending, then series, template, fold, bin ascending); one that no
// stronger kept candidate has absorbed is kept and absorbs every weaker,
// unabsorbed candidate of its series whose F lies within the tolerance of
// (p/q) F for some 1 <= p, q <= max_ratio:
//     1e6 |q F_b - p F_a| <= 1e6 q tol + ppm p F_a     (exact in int64).
// Reduced and unreduced p/q give the same condition, so only coprime pairs
// are tried.  Per series the candidates are kept sorted by F with a
// next-unabsorbed skip array, so each ratio costs one binary search plus the
// candidates it absorbs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "../../include/tb.h"

namespace {

int64_t fundamental(const tb_candidate& c) { return (int64_t)c.bin << (4 - (int)c.log2_harm); }

bool stronger(const tb_candidate& a, const tb_candidate& b)
{
    if (a.sigma != b.sigma) return a.sigma > b.sigma;
    if (a.series_id != b.series_id) return a.series_id < b.series_id;
    if (a.template_id != b.template_id) return a.template_id < b.template_id;
    if (a.log2_harm != b.log2_harm) return a.log2_harm < b.log2_harm;
    return a.bin < b.bin;
}

// Candidates of one series sorted by F; alive(i) = smallest unabsorbed
// position >= i (path-halving skip pointers; size() when none).
struct SeriesIndex {
    std::vector<int64_t> F;
    std::vector<uint32_t> who;
    std::vector<uint32_t> next;

    uint32_t alive(uint32_t i)
    {
        while (next[i] != i) {
            next[i] = next[next[i]];
            i = next[i];
        }
        return i;
    }
    void remove(uint32_t i) { next[i] = i + 1; }
};

int gcd(int a, int b)
{
    while (b) {
        int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

extern "C" tb_status tb_distill(const tb_candidate* in, uint64_t n, uint32_t max_ratio, uint32_t tol,
                                uint32_t ppm, tb_candidate* out, uint32_t* group_size, uint64_t* n_kept)
{
    if (!n_kept || (n && (!in || !out)) || n >= (1ull << 32) || max_ratio < 1 || max_ratio > 64 ||
        tol > (1u << 20) || ppm > 1000000u)
        return TB_ERR_INVALID_ARG;
    for (uint64_t i = 0; i < n; ++i)
        if (in[i].log2_harm > 4 || std::isnan(in[i].sigma)) return TB_ERR_INVALID_ARG;
    const uint32_t N = (uint32_t)n;

    std::vector<uint32_t> order(N);
    std::iota(order.begin(), order.end(), 0u);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return stronger(in[a], in[b]); });

    // per-series indexes; where[i] = (series slot, position in it)
    std::unordered_map<uint32_t, uint32_t> slot_of;
    std::vector<SeriesIndex> ser;
    std::vector<std::pair<uint32_t, uint32_t>> where(N);
    {
        std::vector<uint32_t> cnt;
        std::vector<uint32_t> slot(N);
        for (uint32_t i = 0; i < N; ++i) {
            auto it = slot_of.emplace(in[i].series_id, (uint32_t)cnt.size());
            if (it.second) cnt.push_back(0);
            slot[i] = it.first->second;
            ++cnt[slot[i]];
        }
        ser.resize(cnt.size());
        std::vector<std::vector<uint32_t>> members(cnt.size());
        for (size_t s = 0; s < cnt.size(); ++s) members[s].reserve(cnt[s]);
        for (uint32_t i = 0; i < N; ++i) members[slot[i]].push_back(i);
        for (size_t s = 0; s < cnt.size(); ++s) {
            auto& m = members[s];
            std::sort(m.begin(), m.end(), [&](uint32_t a, uint32_t b) {
                const int64_t fa = fundamental(in[a]), fb = fundamental(in[b]);
                return fa != fb ? fa < fb : a < b;
            });
            SeriesIndex& S = ser[s];
            S.F.resize(m.size());
            S.who = m;
            S.next.resize(m.size() + 1);
            for (uint32_t j = 0; j < (uint32_t)m.size(); ++j) {
                S.F[j] = fundamental(in[m[j]]);
                S.next[j] = j;
                where[m[j]] = {(uint32_t)s, j};
            }
            S.next[m.size()] = (uint32_t)m.size();
        }
    }

    std::vector<std::pair<int, int>> ratios;
    for (int p = 1; p <= (int)max_ratio; ++p)
        for (int q = 1; q <= (int)max_ratio; ++q)
            if (gcd(p, q) == 1) ratios.emplace_back(p, q);

    std::vector<char> decided(N, 0);
    uint64_t kept = 0;
    for (uint32_t a : order) {
        if (decided[a]) continue;
        decided[a] = 1;
        SeriesIndex& S = ser[where[a].first];
        S.remove(where[a].second);
        uint32_t members = 1;
        const int64_t fa = fundamental(in[a]);
        for (const auto& pq : ratios) {
            const int64_t p = pq.first, q = pq.second;
            // |q F_b - p F_a| <= dmax, dmax = floor((1e6 q tol + ppm p F_a) / 1e6)
            const int64_t dmax = (1000000 * q * (int64_t)tol + (int64_t)ppm * p * fa) / 1000000;
            const int64_t lo_num = p * fa - dmax, hi_num = p * fa + dmax;
            const int64_t lo = lo_num <= 0 ? 0 : (lo_num + q - 1) / q;
            const int64_t hi = hi_num / q;
            if (hi < lo) continue;
            uint32_t j = (uint32_t)(std::lower_bound(S.F.begin(), S.F.end(), lo) - S.F.begin());
            for (j = S.alive(j); j < (uint32_t)S.F.size() && S.F[j] <= hi; j = S.alive(j)) {
                decided[S.who[j]] = 1;
                S.remove(j);
                ++members;
            }
        }
        out[kept] = in[a];
        if (group_size) group_size[kept] = members;
        ++kept;
    }
    *n_kept = kept;
    return TB_OK;
}
