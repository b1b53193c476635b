// Host-side planning of a batched launch (no device code, no HIP calls):
// the argument checks of a plan, the largest-first graph order, the team
// configuration of every graph and the device metadata image.  Shared by
// the batched plans, the server and the CPU tests (which run it under
// AddressSanitizer).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <utility>
#include <vector>

#include "apsp.h"

namespace apsp {

constexpr int kBatchBS = 64;         // graphs with n <= 64 are solved by one wavefront
constexpr int kBatchThreads = 256;   // threads of a batched workgroup
constexpr int kBatchMaxN = 1024;     // largest graph of a batch
enum TeamCfg { kWaveTiles64 = 0, kGroupTiles64 = 1, kGroupTiles128 = 2, kMixed128 = 3 };

// Size classes of the tuning table: n in (64,128], (128,192], ..., (448,512]
// (64 wide, so a class pads its graphs to one multiple of 64) and (512,1024].
constexpr int kClasses = 8;
constexpr int kClassHi[kClasses] = {128, 192, 256, 320, 384, 448, 512, 1024};

inline int size_class(int64_t n) {
    for (int c = 0; c < kClasses; ++c)
        if (n <= kClassHi[c]) return c;
    return kClasses - 1;
}

// Padding granularity of a team configuration in the general kernel.
inline int team_bs(int cfg) { return cfg == kGroupTiles128 ? 128 : 64; }

// Arguments of a plan: sizes 1..kBatchMaxN, offsets multiples of 4 and
// non-negative, forced configurations in -1..kMixed128, graphs pairwise
// disjoint.  *max_end receives the elements the packed buffers must hold.
inline apsp_status_t plan_args_check(const int32_t *ns, const int64_t *offsets, int32_t batch,
                                     const int8_t *team_config, int64_t *max_end) {
    if (batch < 0 || (batch > 0 && (!ns || !offsets))) return APSP_ERROR_INVALID_ARGUMENT;
    int64_t end_max = 0;
    std::vector<std::pair<int64_t, int64_t>> spans;
    spans.reserve((size_t)batch);
    for (int32_t b = 0; b < batch; ++b) {
        if (ns[b] < 1 || ns[b] > kBatchMaxN || offsets[b] < 0 || offsets[b] % 4 != 0)
            return APSP_ERROR_INVALID_ARGUMENT;
        if (team_config && (team_config[b] < -1 || team_config[b] > kMixed128)) return APSP_ERROR_INVALID_ARGUMENT;
        const int64_t end = offsets[b] + (int64_t)ns[b] * ns[b];
        end_max = std::max(end_max, end);
        spans.push_back({offsets[b], end});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return APSP_ERROR_INVALID_ARGUMENT;  // overlap
    if (max_end) *max_end = end_max;
    return APSP_SUCCESS;
}

// Graph ids, largest n first (stable); order[0, n_team) have n > kBatchBS.
inline void batch_order(const int32_t *ns, int32_t batch, std::vector<int32_t> &order, int32_t &n_team) {
    order.resize((size_t)batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ns[a] > ns[b]; });
    n_team = 0;
    while (n_team < batch && ns[order[(size_t)n_team]] > kBatchBS) ++n_team;
}

// Host image of a batch's device metadata:
//   order[B] int32 | ns[B] int32 | offsets[B] int64 | cfg[B] int8
// with the team configuration of every graph (forced, or cfg_of(n)), and the
// work-matrix elements one workgroup needs.
//
// lean (out): the batch runs in the lean distance kernel, which takes the
// graphs above 64 vertices when every one of them has configuration
// kMixed128 or kGroupTiles64 (work matrices padded to 64) and there are no
// predecessors; otherwise the general kernel runs, which solves kMixed128
// graphs as kGroupTiles128 (padded to 128).
template <class CfgOf>
void batch_meta_with(const int32_t *ns, const int64_t *offsets, int32_t B, bool pred, const int8_t *forced,
                     CfgOf cfg_of, std::vector<char> &bytes, int32_t &n_team, int64_t &scratch_elems,
                     bool &lean) {
    std::vector<int32_t> order;
    batch_order(ns, B, order, n_team);
    bytes.assign(std::max<size_t>((size_t)B * 17 + 16, 32), 0);
    std::copy(order.begin(), order.end(), (int32_t *)bytes.data());
    std::copy(ns, ns + B, (int32_t *)bytes.data() + B);
    std::copy(offsets, offsets + B, (int64_t *)(bytes.data() + (size_t)B * 8));
    int8_t *cfg = (int8_t *)(bytes.data() + (size_t)B * 16);
    lean = !pred;
    for (int32_t b = 0; b < B; ++b) {
        const int8_t c = forced && forced[b] >= 0 ? forced[b] : (int8_t)cfg_of(ns[b]);
        cfg[b] = c;
        if (ns[b] > kBatchBS && c != kMixed128 && c != kGroupTiles64) lean = false;
    }
    scratch_elems = 0;
    for (int32_t b = 0; b < B; ++b) {
        if (!lean && cfg[b] == kMixed128) cfg[b] = kGroupTiles128;
        if (ns[b] > kBatchBS) {
            const int64_t bs = lean ? 64 : team_bs(cfg[b]), ldp = (ns[b] + bs - 1) / bs * bs;
            scratch_elems = std::max(scratch_elems, ldp * ldp);
        }
    }
}

}  // namespace apsp
