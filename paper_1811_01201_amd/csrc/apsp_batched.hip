// Batched blocked Floyd–Warshall: many independent graphs of uneven size in
// one persistent, fused launch.
//
// Each 256-thread workgroup (four wavefronts) loops, pulling work from a
// device counter, graphs ordered largest first:
//   * a graph with n > 64 is solved by the whole workgroup: it is copied
//     into the workgroup's private work matrix (padded to a multiple of 64
//     with isolated vertices), then the paper's rounds (Section "Data
//     Locality") run with 64-wide k-blocks: wavefront 0 closes the diagonal
//     block, the four wavefronts share the block-row/block-column tiles and
//     then the remaining tiles (64 x 64 each, one wavefront per tile, no
//     workgroup barrier inside a tile), and the result is copied back;
//   * once those are exhausted each wavefront pulls graphs with n <= 64 on
//     its own and closes them entirely in registers (n k-steps).
// The last workgroup to finish resets the counters, so the plan can be
// replayed (also from a captured hipGraph) without a separate reset launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "apsp_batch_host.h"
#include "apsp_internal.h"

namespace apsp {

struct BatchMeta {
    const int32_t *order;    // graph ids, largest n first
    const int32_t *ns;       // n of each graph
    const int64_t *offsets;  // element offset of each graph in the packed buffers
    const int8_t *cfg;       // team configuration of each graph
    int32_t batch;
    int32_t n_team;          // order[0, n_team) have n > 64
    int64_t scratch_elems;   // work-matrix elements per workgroup
};


// ------------------------------------------------ input/output conversion
template <class Ar, class Tin>
__device__ __forceinline__ typename Ar::T to_work(const Ar &ar, Tin w, bool inside, int64_t i,
                                                  int64_t j) {
    bool absent;
    if (!inside)
        absent = (i != j);
    else if constexpr (std::is_same_v<Tin, int32_t>)
        absent = (w == kInf32);
    else
        absent = (w == __builtin_inff());
    const bool edge = !absent && i != j;
    const double x = inside ? (double)w : 0.0;
    if constexpr (std::is_same_v<Ar, ArI32>) {
        return absent ? kInf32 : (int32_t)x;
    } else if constexpr (std::is_same_v<Ar, ArF32>) {
        return absent ? __builtin_inff() : (float)x;
    } else if constexpr (std::is_same_v<Ar, ArKey>) {
        const double none = (double)((1 << ar.S) - 1);
        return absent ? __builtin_inf() : __builtin_ldexp(x, ar.S) + (edge ? (double)i : none);
    } else {
        return DistPred{absent ? __builtin_inff() : (float)x, edge ? (int32_t)i : kLexNone};
    }
}

// Writes distance (and predecessor) of one element; returns true for a
// negative diagonal entry.
template <class Ar, class Tin>
__device__ __forceinline__ bool from_work(const Ar &ar, typename Ar::T v, int64_t i, int64_t j,
                                          Tin *d, int32_t *p) {
    constexpr Tin inf = std::is_same_v<Tin, int32_t> ? Tin(kInf32) : Tin(__builtin_huge_valf());
    bool neg = false;
    int32_t pr = APSP_NO_PRED;
    Tin out;
    if constexpr (std::is_same_v<Ar, ArI32>) {
        out = v >= kFakeThreshold ? kInf32 : v;
        neg = ((i == j) && v < 0) || v < kWrapWitness;
    } else if constexpr (std::is_same_v<Ar, ArF32>) {
        if constexpr (std::is_same_v<Tin, int32_t>)  // int32 weights solved in float32 (exact)
            out = (v == __builtin_inff()) ? kInf32 : (int32_t)v;
        else
            out = v;
        neg = (i == j) && v < 0.0f;
    } else if constexpr (std::is_same_v<Ar, ArKey>) {
        if (v == __builtin_inf()) {
            out = inf;
        } else {
            const double dd = __builtin_floor(__builtin_ldexp(v, -ar.S));
            pr = (int32_t)(v - __builtin_ldexp(dd, ar.S));
            if (pr == (1 << ar.S) - 1) pr = APSP_NO_PRED;
            out = (Tin)dd;
            neg = (i == j) && dd < 0.0;
        }
    } else {
        if (v.d == __builtin_inff()) {
            out = inf;
        } else {
            out = (Tin)v.d;
            pr = (v.p == kLexNone) ? APSP_NO_PRED : v.p;
            neg = (i == j) && v.d < 0.0f;
        }
    }
    if (i == j) pr = APSP_NO_PRED;
    *d = out;
    if (p) *p = pr;
    return neg;
}

// ------------------------------------------- per-graph policy choice
// A graph takes the second policy Alt when one of its weights rules out the
// first:
//   float32 weights with predecessors (ArKey / ArLexF32): a finite weight
//     that is not an integer within the bound (keys would not be exact);
//   int32 distances (ArF32 / ArI32): a negative weight or one with
//     |w| (n - 1) >= 2^23.  Otherwise every operand the blocked schedule
//     adds is a restricted shortest-path length below 2^23 in magnitude, so
//     every float32 sum is an exact integer below 2^24 and the float32
//     solve equals the int32 one; float32 adds issue at twice the rate.
// The int32 test as one unsigned comparison: w (n - 1) >= 2^23 for w >= 0
// is w >= lim = ceil(2^23 / (n - 1)), and a negative w read as unsigned is
// at least 2^31 > lim.  n <= 1: lim = 2^31 (only negative weights).
__device__ __forceinline__ uint32_t f32_limit(int64_t n) {
    return n <= 1 ? 0x80000000u : (uint32_t)(((int64_t(1) << 23) + (n - 2)) / (n - 1));
}
__device__ __forceinline__ bool f32_ruled_out(int32_t w, uint32_t lim) {
    return ((uint32_t)w >= lim) & (w != kInf32);
}

// Per-graph form of the test: lim() once per graph, out() per weight.
template <class Ar, class Alt, class Tin>
struct RuleOut {
    float bound;
    __device__ __forceinline__ explicit RuleOut(int64_t n) : bound((float)weight_bound(n)) {}
    __device__ __forceinline__ bool out(Tin w) const {
        const float f = (float)w;
        return (f != __builtin_inff()) & ((f != __builtin_floorf(f)) | (__builtin_fabsf(f) > bound));
    }
};
template <>
struct RuleOut<ArF32, ArI32, int32_t> {
    uint32_t lim;
    __device__ __forceinline__ explicit RuleOut(int64_t n) : lim(f32_limit(n)) {}
    __device__ __forceinline__ bool out(int32_t w) const { return f32_ruled_out(w, lim); }
};

// ------------------------------------------------------------ team path
// Team configurations (chosen per graph; see the plan's size classes):
//   kWaveTiles64   64-wide k-blocks; each wavefront owns whole 64 x 64 tiles
//                  (8 x 8 registers per lane, no workgroup barrier inside a
//                  tile); the whole workgroup closes the diagonal block
//                  (4 x 4 per thread: measured 7-16 % faster per graph than
//                  leaving it to one wavefront)
//   kGroupTiles64  64-wide k-blocks; the workgroup works on one 64 x 64 tile
//                  at a time (4 x 4 registers per thread) and closes the
//                  diagonal block together (4 x 4 per thread)
//   kGroupTiles128 128-wide k-blocks; 128 x 128 workgroup tiles (8 x 8 per
//                  thread), diagonal block closed by the workgroup
template <class Ar>
using BTile = TileProduct<Ar, kBatchBS, kBatchBS, (sizeof(typename Ar::T) == 4 ? 16 : 8), 8, 8, true>;
template <class Ar>
using GTile64 = std::conditional_t<sizeof(typename Ar::T) == 4, TileProductDMA<Ar, 64, 64, 16, 4, 4>,
                                   TileProduct<Ar, 64, 64, 16, 4, 4>>;
template <class Ar>
using GTile128 = std::conditional_t<sizeof(typename Ar::T) == 4, TileProductDMA<Ar, 128, 128, 16, 8, 8>,
                                    TileProduct<Ar, 128, 128, 16, 8, 8>>;

template <int CFG>
struct TeamShape {
    static constexpr int BS = CFG == kGroupTiles128 ? 128 : 64;
};

template <class Ar>
union alignas(16) TeamSmem {
    typename BTile<Ar>::Smem wave[kBatchThreads / 64];
    typename GTile64<Ar>::Smem g64;
    typename GTile128<Ar>::Smem g128;
    typename Ar::T p1[8 * 128];  // phase-1 publication buffers (4 column + 4 row)
};

// CHECK: the float32 launch of an int32 batch; the graph is dropped (left
// to the int32 launch) if a weight rules float32 arithmetic out, which the
// copy into the work matrix checks on the way.
template <class Ar, class Tin, int CFG, bool CHECK = false>
__device__ void team_solve(const Ar &ar0, Tin *__restrict__ dist, int32_t *__restrict__ pred,
                           int32_t *__restrict__ status, int g, int64_t n, int64_t off,
                           typename Ar::T *__restrict__ X, TeamSmem<Ar> &sm) {
    using T = typename Ar::T;
    constexpr int BS = TeamShape<CFG>::BS;
    Ar ar = ar0;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int64_t ldp = (n + BS - 1) / BS * BS;
    if constexpr (std::is_same_v<Ar, ArKey>) {
        int S = 1;
        while ((int64_t(1) << S) < ldp + 1) ++S;
        ar.S = S;
    }
    bool ruled_out = false;
    const uint32_t lim = f32_limit(n);
    for (int64_t e = tid; e < ldp * ldp; e += kBatchThreads) {
        const int64_t i = e / ldp, j = e - i * ldp;
        const bool inside = i < n && j < n;
        const Tin w = inside ? dist[off + i * n + j] : Tin(0);
        if constexpr (CHECK) ruled_out |= inside & f32_ruled_out(w, lim);
        X[e] = to_work(ar, w, inside, i, j);
    }
    if constexpr (CHECK) {
        if (__syncthreads_or(ruled_out)) return;  // uniform: the whole workgroup leaves
    } else {
        __syncthreads();
    }
    const int R = (int)(ldp / BS);
    const int nt = R - 1;
    T(*buf)[BS] = reinterpret_cast<T(*)[BS]>(sm.p1);
    for (int r = 0; r < R; ++r) {
        const int64_t r0 = (int64_t)r * BS;
        // the last block's k-range stops at n, rounded up to 32 (whole pairs
        // of 16-wide chunks): the vertices beyond n are isolated padding
        const int kc = r + 1 < R ? BS : (int)((n - r0 + 31) / 32 * 32);
        // phase 1
        if constexpr (CFG == kGroupTiles128)
            phase1_body<Ar, 128, false, 8>(X, ldp, r0, ar, buf, buf + 4, kc);
        else
            phase1_body<Ar, 64, false, 4>(X, ldp, r0, ar, buf, buf + 4, kc);
        __syncthreads();
        // phase 2: block row r (tiles t < nt) and block column r
        if constexpr (CFG == kWaveTiles64) {
            for (int t = wave; t < 2 * nt; t += kBatchThreads / 64) {
                const bool is_row = t < nt;
                int q = is_row ? t : t - nt;
                q += (q >= r) ? 1 : 0;
                const int64_t o = (int64_t)q * BS;
                if (is_row)
                    BTile<Ar>::run(sm.wave[wave], X, ldp, r0, o, r0, kc, ar);
                else
                    BTile<Ar>::run(sm.wave[wave], X, ldp, o, r0, r0, kc, ar);
            }
        } else {
            for (int t = 0; t < 2 * nt; ++t) {
                const bool is_row = t < nt;
                int q = is_row ? t : t - nt;
                q += (q >= r) ? 1 : 0;
                const int64_t o = (int64_t)q * BS;
                const int64_t crow = is_row ? r0 : o, ccol = is_row ? o : r0;
                if constexpr (CFG == kGroupTiles64)
                    GTile64<Ar>::run(sm.g64, X, ldp, crow, ccol, r0, kc, ar);
                else
                    GTile128<Ar>::run(sm.g128, X, ldp, crow, ccol, r0, kc, ar);
            }
        }
        __syncthreads();
        // phase 3: every other tile
        if constexpr (CFG == kWaveTiles64) {
            for (int t = wave; t < nt * nt; t += kBatchThreads / 64) {
                int ti = t / nt, tj = t - (t / nt) * nt;
                ti += (ti >= r) ? 1 : 0;
                tj += (tj >= r) ? 1 : 0;
                BTile<Ar>::run(sm.wave[wave], X, ldp, (int64_t)ti * BS, (int64_t)tj * BS, r0, kc, ar);
            }
        } else {
            for (int t = 0; t < nt * nt; ++t) {
                int ti = t / nt, tj = t - (t / nt) * nt;
                ti += (ti >= r) ? 1 : 0;
                tj += (tj >= r) ? 1 : 0;
                if constexpr (CFG == kGroupTiles64)
                    GTile64<Ar>::run(sm.g64, X, ldp, (int64_t)ti * BS, (int64_t)tj * BS, r0, kc, ar);
                else
                    GTile128<Ar>::run(sm.g128, X, ldp, (int64_t)ti * BS, (int64_t)tj * BS, r0, kc, ar);
            }
        }
        __syncthreads();
    }
    bool neg = false;
    for (int64_t e = tid; e < n * n; e += kBatchThreads) {
        const int64_t i = e / n, j = e - i * n;
        neg |= from_work(ar, X[i * ldp + j], i, j, dist + off + e, pred ? pred + off + e : nullptr);
    }
    neg = __syncthreads_or(neg);
    if (status && tid == 0) status[g] = neg ? APSP_ERROR_NEGATIVE_CYCLE : APSP_SUCCESS;
    __syncthreads();
}

template <class Ar, class Tin, bool CHECK = false>
__device__ void team_dispatch(int cfg, const Ar &ar, Tin *__restrict__ dist, int32_t *__restrict__ pred,
                              int32_t *__restrict__ status, int g, int64_t n, int64_t off,
                              typename Ar::T *__restrict__ X, TeamSmem<Ar> &sm) {
    if (cfg == kGroupTiles64)
        team_solve<Ar, Tin, kGroupTiles64, CHECK>(ar, dist, pred, status, g, n, off, X, sm);
    else if (cfg == kGroupTiles128)
        team_solve<Ar, Tin, kGroupTiles128, CHECK>(ar, dist, pred, status, g, n, off, X, sm);
    else
        team_solve<Ar, Tin, kWaveTiles64, CHECK>(ar, dist, pred, status, g, n, off, X, sm);
}

// ------------------------------------------------------ wavefront path
// n <= 64: the whole graph in one wavefront's registers (8 x 8 per lane).
// CHECK as for team_solve.
template <class Ar, class Tin, bool CHECK = false>
__device__ __forceinline__ bool wave_solve(const Ar &ar0, Tin *__restrict__ dist, int32_t *__restrict__ pred,
                           int32_t *__restrict__ status, int g, int64_t n, int64_t off,
                           typename Ar::T (*colbuf)[kBatchBS], typename Ar::T (*rowbuf)[kBatchBS]) {
    using T = typename Ar::T;
    Ar ar = ar0;
    if constexpr (std::is_same_v<Ar, ArKey>) ar.S = 7;  // vertices 0..63, none = 127
    const int lane = threadIdx.x & 63, tx = lane % 8, ty = lane / 8;
    T c[8][8];
    bool ruled_out = false;
    const uint32_t lim = f32_limit(n);
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = ty * 8 + m, j = tx * 8 + q;
            const bool inside = i < n && j < n;
            const Tin w = inside ? dist[off + i * n + j] : Tin(0);
            if constexpr (CHECK) ruled_out |= inside & f32_ruled_out(w, lim);
            c[m][q] = to_work(ar, w, inside, i, j);
        }
    if constexpr (CHECK) {
        if (__any(ruled_out)) return false;  // uniform over the wavefront
    }
    const int ksteps = (int)((n + 15) / 16 * 16);  // vertices >= n are isolated
    phase1_steps<Ar, kBatchBS, true>(c, ksteps, ar, colbuf, rowbuf);
    bool neg = false;
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = ty * 8 + m, j = tx * 8 + q;
            if (i < n && j < n)
                neg |= from_work(ar, c[m][q], i, j, dist + off + i * n + j,
                                 pred ? pred + off + i * n + j : nullptr);
        }
    neg = __any(neg);
    if (status && lane == 0) status[g] = neg ? APSP_ERROR_NEGATIVE_CYCLE : APSP_SUCCESS;
    return true;
}

// Whether any weight of a graph (count elements from a 16-byte-aligned g)
// rules out policy Ar in favour of Alt: 16-byte loads, several in flight
// per lane, lanes lane, lane + width, ... of the caller's group.
template <class Ar, class Alt, class Tin>
__device__ __forceinline__ bool scan_rules_out(const Tin *__restrict__ g, int64_t count, int64_t n, int lane,
                                               int width) {
    const RuleOut<Ar, Alt, Tin> rule(n);
    const int64_t nv = count / 4;
    const int4 *__restrict__ v = reinterpret_cast<const int4 *>(g);
    auto any4 = [&](const int4 &x) {
        Tin a[4];
        __builtin_memcpy(a, &x, 16);
        return rule.out(a[0]) | rule.out(a[1]) | rule.out(a[2]) | rule.out(a[3]);
    };
    bool out = false;
    int64_t e = lane;
    // eight 16-byte loads in flight per lane, then their tests
    for (; e + 7 * (int64_t)width < nv; e += 8 * (int64_t)width) {
        int4 x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = v[e + u * (int64_t)width];
#pragma unroll
        for (int u = 0; u < 8; ++u) out |= any4(x[u]);
    }
    for (; e < nv; e += width) out |= any4(v[e]);
    for (int64_t t = nv * 4 + lane; t < count; t += width) out |= rule.out(g[t]);
    return out;
}

// ------------------------------------------------------------- the kernel
// counters[0]: next team graph, [1]: next wavefront graph, [2]: finished
// workgroups.  With a second policy Alt, each graph is checked first and
// solved with Alt when rules_out says so.  SEL splits int32 distance
// batches over two launches with one arithmetic each (a kernel holding
// both spills registers): kIntGraphs solves only the graphs rules_out
// excludes from float32 arithmetic, kFloatGraphs only the others.  The
// int32 launch runs first, so the float32 one still sees the weights of
// the graphs it solves; a graph the int32 launch solved may pass the check
// afterwards and be solved again from its distances, which leaves them
// unchanged.
enum BatchSel { kEveryGraph = 0, kIntGraphs = 1, kFloatGraphs = 2 };

template <int SEL, class Tin>
__device__ __forceinline__ bool selected(bool excluded_from_float) {
    if constexpr (SEL == kIntGraphs) return excluded_from_float;
    if constexpr (SEL == kFloatGraphs) return !excluded_from_float;
    return true;
}

template <class Tin, class Ar, class Alt, int SEL>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(2)))
batched_kernel(BatchMeta meta, Tin *__restrict__ dist, int32_t *__restrict__ pred,
               int32_t *__restrict__ status, void *__restrict__ scratch, int32_t *__restrict__ counters,
               Ar ar, Alt alt) {
    constexpr bool kDual = !std::is_same_v<Alt, NoAlt>;
    __shared__ union {
        TeamSmem<Ar> a;
        TeamSmem<std::conditional_t<kDual, Alt, Ar>> b;
    } sm;
    __shared__ int s_q;
    const int tid = threadIdx.x;
    char *const my_scratch = (char *)scratch + (int64_t)blockIdx.x * meta.scratch_elems *
                                                   std::max(sizeof(typename Ar::T),
                                                            sizeof(typename Alt::T));
    for (;;) {
        if (tid == 0) s_q = atomicAdd(&counters[0], 1);
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= meta.n_team) break;
        const int g = meta.order[q];
        const int64_t n = meta.ns[g], off = meta.offsets[g];
        if constexpr (SEL == kIntGraphs) {
            const bool out = scan_rules_out<ArF32, ArI32>(dist + off, n * n, n, tid, kBatchThreads);
            if (!selected<SEL, Tin>(__syncthreads_or(out))) continue;
        }
        bool use_alt = false;
        if constexpr (kDual) {
            use_alt = __syncthreads_or(scan_rules_out<Ar, Alt>(dist + off, n * n, n, tid, kBatchThreads));
        }
        const int cfg = meta.cfg[g];
        if constexpr (kDual) {
            if (use_alt) {
                team_dispatch<Alt, Tin>(cfg, alt, dist, pred, status, g, n, off,
                                        (typename Alt::T *)my_scratch, sm.b);
                continue;
            }
        }
        // the float32 launch checks the weights while copying them in
        team_dispatch<Ar, Tin, SEL == kFloatGraphs>(cfg, ar, dist, pred, status, g, n, off,
                                                    (typename Ar::T *)my_scratch, sm.a);
    }
    // small graphs: every wavefront on its own
    const int wave = tid >> 6, lane = tid & 63;
    for (;;) {
        int q = 0;
        if (lane == 0) q = atomicAdd(&counters[1], 1);
        q = __shfl(q, 0) + meta.n_team;
        if (q >= meta.batch) break;
        const int g = meta.order[q];
        const int64_t n = meta.ns[g], off = meta.offsets[g];
        if constexpr (SEL == kIntGraphs) {
            const bool out = scan_rules_out<ArF32, ArI32>(dist + off, n * n, n, lane, 64);
            if (!selected<SEL, Tin>(__any(out))) continue;
        }
        bool use_alt = false;
        if constexpr (kDual) {
            use_alt = __any(scan_rules_out<Ar, Alt>(dist + off, n * n, n, lane, 64));
        }
        if constexpr (kDual) {
            if (use_alt) {
                using TA = typename Alt::T;
                TA(*buf)[kBatchBS] = reinterpret_cast<TA(*)[kBatchBS]>(&sm.b.wave[wave]);
                wave_solve<Alt, Tin>(alt, dist, pred, status, g, n, off, buf, buf + 4);
                continue;
            }
        }
        using TR = typename Ar::T;
        TR(*buf)[kBatchBS] = reinterpret_cast<TR(*)[kBatchBS]>(&sm.a.wave[wave]);
        wave_solve<Ar, Tin, SEL == kFloatGraphs>(ar, dist, pred, status, g, n, off, buf, buf + 4);
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&counters[2], 1) == (int)gridDim.x - 1) {
            counters[0] = 0;
            counters[1] = 0;
            counters[2] = 0;
            __threadfence();
        }
    }
}


// ------------------------------------------------------ lean distance launch
// Distance batches whose graphs above 64 vertices all take the padded-to-64
// team path below run in a kernel that holds nothing else (plus the
// one-wavefront path for n <= 64), so its register budget is that of one
// 128 x 128 tile product: no scratch spills and three workgroups per CU.
//
// kMixed128: the work matrix is padded to a multiple of 64 (not 128); the
// k-blocks are 128 wide except the last, which is 64 wide when the padded
// order is an odd multiple of 64, and the C tiles follow the blocks, so a
// tile is 128 or 64 rows by 128 or 64 columns.  Every tile is one
// workgroup product with the A and B chunks brought into LDS by DMA.  In
// the last round the k-range stops at n rounded up to 32 (the vertices
// beyond n are isolated padding).  kGroupTiles64 runs the same code with
// 64-wide blocks only.  Both arithmetics of an int32 batch are in the
// kernel: the graph is copied in as float32 while its weights are checked,
// and copied again and solved in int32 when a weight rules float32 out.
template <class Ar>
using LT11 = TileProductDMA<Ar, 128, 128, 16, 8, 8>;
template <class Ar>
using LT10 = TileProductDMA<Ar, 128, 64, 16, 8, 4>;
template <class Ar>
using LT01 = TileProductDMA<Ar, 64, 128, 16, 4, 8>;
template <class Ar>
using LT00 = TileProductDMA<Ar, 64, 64, 16, 4, 4>;

// LDS of the lean kernel: four distinct chunk buffers shared by every tile
// shape (distinct arrays, so the compiler keeps a chunk copy in flight
// while the other buffer is read), the phase-1 publications and the
// one-wavefront path's buffers.
constexpr int kLeanChunk = 128 * 16;  // elements of the largest A or B chunk
template <class T>
struct LeanLds {
    T *a0, *a1, *b0, *b1;
    T *p1;    // 8 x 128: 4 column + 4 row publications
    T *wave;  // 4 wavefronts x 8 x 64
};

// C (h x w at crow, ccol) <- min(C, A (h x kc at crow, k0) (x) B (kc x w at k0, ccol)); h, w in {64, 128}
template <class Ar>
__device__ __forceinline__ void lean_tile(const LeanLds<typename Ar::T> &sm, typename Ar::T *X, int64_t ldp,
                                          int64_t crow, int64_t ccol, int h, int w, int64_t k0, int kc,
                                          const Ar &ar) {
    if (h == 128) {
        if (w == 128)
            LT11<Ar>::run_in(sm.a0, sm.a1, sm.b0, sm.b1, X, ldp, crow, ccol, k0, kc, ar);
        else
            LT10<Ar>::run_in(sm.a0, sm.a1, sm.b0, sm.b1, X, ldp, crow, ccol, k0, kc, ar);
    } else {
        if (w == 128)
            LT01<Ar>::run_in(sm.a0, sm.a1, sm.b0, sm.b1, X, ldp, crow, ccol, k0, kc, ar);
        else
            LT00<Ar>::run_in(sm.a0, sm.a1, sm.b0, sm.b1, X, ldp, crow, ccol, k0, kc, ar);
    }
}

// Copies graph (n x n at src, leading dimension n) into X (ldp x ldp) in the
// policy's form, padding vertices isolated; CHECK: returns, uniformly over
// the workgroup, whether a weight rules float32 arithmetic out.
template <class Ar, class Tin, bool CHECK>
__device__ __forceinline__ bool lean_copy_in(const Ar &ar, const Tin *__restrict__ src, int n, int ldp,
                                             typename Ar::T *__restrict__ X) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool ruled_out = false;
    const uint32_t lim = f32_limit(n);
    // one row per wavefront at a time, all of its loads issued before the
    // first is used (a row has at most 16 64-wide pieces)
    for (int i = wave; i < ldp; i += kBatchThreads / 64) {
        for (int j0 = 0; j0 < ldp; j0 += 16 * 64) {
            Tin w[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = j0 + t * 64 + lane;
                w[t] = (i < n && j < n) ? src[(uint32_t)i * (uint32_t)n + (uint32_t)j] : Tin(0);
            }
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = j0 + t * 64 + lane;
                const bool inside = i < n && j < n;
                if constexpr (CHECK) ruled_out |= inside & f32_ruled_out(w[t], lim);
                if (j < ldp) X[(uint32_t)i * (uint32_t)ldp + (uint32_t)j] = to_work(ar, w[t], inside, i, j);
            }
        }
    }
    if constexpr (CHECK) return __syncthreads_or(ruled_out);
    __syncthreads();
    return false;
}

// The rounds of one graph on X (ldp x ldp, ldp a multiple of 64); BMAX is
// the block width (128: kMixed128, 64: kGroupTiles64).
template <class Ar, int BMAX>
__device__ __forceinline__ void lean_rounds(const Ar &ar, typename Ar::T *__restrict__ X, int n, int ldp,
                                            const LeanLds<typename Ar::T> &sm) {
    using T = typename Ar::T;
    const int R = (ldp + BMAX - 1) / BMAX;
    auto width = [&](int q) { return min(BMAX, ldp - q * BMAX); };
    for (int r = 0; r < R; ++r) {
        const int r0 = r * BMAX, wr = width(r);
        // the last block's k-range stops at n, rounded up to 32 (whole pairs
        // of 16-wide chunks): the vertices beyond n are isolated padding
        const int kc = r + 1 < R ? wr : min(wr, (n - r0 + 31) / 32 * 32);
        if (BMAX == 128 && wr == 128)
            phase1_body<Ar, 128, false, 8>(X, ldp, r0, ar, reinterpret_cast<T(*)[128]>(sm.p1),
                                           reinterpret_cast<T(*)[128]>(sm.p1) + 4, kc);
        else
            phase1_body<Ar, 64, false, 4>(X, ldp, r0, ar, reinterpret_cast<T(*)[64]>(sm.p1),
                                          reinterpret_cast<T(*)[64]>(sm.p1) + 4, kc);
        __syncthreads();
        // phase 2: block row r against the closed diagonal block (A = that
        // block, B = the tile itself) and block column r (A = the tile
        // itself, B = the block); each tile spans the whole block in the
        // direction it reads from itself
        for (int q = 0; q < R; ++q) {
            if (q == r) continue;
            const int wq = width(q);
            lean_tile<Ar>(sm, X, ldp, r0, (int64_t)q * BMAX, wr, wq, r0, kc, ar);
            lean_tile<Ar>(sm, X, ldp, (int64_t)q * BMAX, r0, wq, wr, r0, kc, ar);
        }
        __syncthreads();
        // phase 3: every other tile from its row's and column's panel tiles
        for (int p = 0; p < R; ++p) {
            if (p == r) continue;
            for (int q = 0; q < R; ++q) {
                if (q == r) continue;
                lean_tile<Ar>(sm, X, ldp, (int64_t)p * BMAX, (int64_t)q * BMAX, width(p), width(q), r0, kc, ar);
            }
        }
        __syncthreads();
    }
}

// Writes graph g's result from X, and its status.
template <class Ar, class Tin>
__device__ __forceinline__ void lean_copy_out(const Ar &ar, const typename Ar::T *__restrict__ X, int n, int ldp,
                                              Tin *__restrict__ dst, int32_t *__restrict__ status, int g) {
    using T = typename Ar::T;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool neg = false;
    for (int i = wave; i < n; i += kBatchThreads / 64) {
        for (int j0 = 0; j0 < n; j0 += 16 * 64) {
            T v[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = j0 + t * 64 + lane;
                v[t] = j < n ? X[(uint32_t)i * (uint32_t)ldp + (uint32_t)j] : T(0);
            }
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = j0 + t * 64 + lane;
                if (j < n)
                    neg |= from_work(ar, v[t], i, j, dst + ((uint32_t)i * (uint32_t)n + (uint32_t)j),
                                     (int32_t *)nullptr);
            }
        }
    }
    neg = __syncthreads_or(neg);
    if (status && threadIdx.x == 0) status[g] = neg ? APSP_ERROR_NEGATIVE_CYCLE : APSP_SUCCESS;
    __syncthreads();
}

// One team graph: Ar first (checked against Alt's rule when Alt is not
// NoAlt), Alt when a weight rules Ar out.
template <class Tin, class Ar, class Alt, int BMAX>
__device__ __forceinline__ void lean_team(const Ar &ar, const Alt &alt, Tin *__restrict__ dist,
                                          int32_t *__restrict__ status, int g, int n, int64_t off, void *scratch,
                                          const LeanLds<typename Ar::T> &sm) {
    constexpr bool kDual = !std::is_same_v<Alt, NoAlt>;
    const int ldp = (n + 63) / 64 * 64;
    Tin *const src = dist + off;
    typename Ar::T *const X = (typename Ar::T *)scratch;
    if (!lean_copy_in<Ar, Tin, kDual>(ar, src, n, ldp, X)) {
        lean_rounds<Ar, BMAX>(ar, X, n, ldp, sm);
        lean_copy_out<Ar, Tin>(ar, X, n, ldp, src, status, g);
        return;
    }
    if constexpr (kDual) {
        static_assert(sizeof(typename Alt::T) == sizeof(typename Ar::T), "one work-matrix layout");
        using TA = typename Alt::T;
        typename Alt::T *const Y = (TA *)scratch;
        const LeanLds<TA> sa{(TA *)sm.a0, (TA *)sm.a1, (TA *)sm.b0, (TA *)sm.b1, (TA *)sm.p1, (TA *)sm.wave};
        lean_copy_in<Alt, Tin, false>(alt, src, n, ldp, Y);
        lean_rounds<Alt, BMAX>(alt, Y, n, ldp, sa);
        lean_copy_out<Alt, Tin>(alt, Y, n, ldp, src, status, g);
    }
}

// counters[0]: next team graph, [1]: next wavefront graph, [2]: finished
// workgroups (the last one resets all three).  Distances only.
template <class Tin, class Ar, class Alt>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(3)))
batched_lean_kernel(BatchMeta meta, Tin *__restrict__ dist, int32_t *__restrict__ status,
                    void *__restrict__ scratch, int32_t *__restrict__ counters, Ar ar, Alt alt) {
    static_assert(sizeof(typename Ar::T) == 4, "distance policies");
    constexpr bool kDual = !std::is_same_v<Alt, NoAlt>;
    using TR = typename Ar::T;
    __shared__ alignas(16) TR la0[kLeanChunk];
    __shared__ alignas(16) TR la1[kLeanChunk];
    __shared__ alignas(16) TR lb0[kLeanChunk];
    __shared__ alignas(16) TR lb1[kLeanChunk];
    __shared__ alignas(16) TR lp1[8 * 128];
    __shared__ alignas(16) TR lwave[4 * 8 * kBatchBS];
    const LeanLds<TR> sm{la0, la1, lb0, lb1, lp1, lwave};
    __shared__ int s_q;
    const int tid = threadIdx.x;
    void *const my_scratch = (char *)scratch + (int64_t)blockIdx.x * meta.scratch_elems * 4;
    for (;;) {
        if (tid == 0) s_q = atomicAdd(&counters[0], 1);
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= meta.n_team) break;
        const int g = meta.order[q];
        const int n = meta.ns[g];
        const int64_t off = meta.offsets[g];
        if (meta.cfg[g] == kGroupTiles64)
            lean_team<Tin, Ar, Alt, 64>(ar, alt, dist, status, g, n, off, my_scratch, sm);
        else
            lean_team<Tin, Ar, Alt, 128>(ar, alt, dist, status, g, n, off, my_scratch, sm);
    }
    // small graphs: every wavefront on its own
    const int wave = tid >> 6, lane = tid & 63;
    for (;;) {
        int q = 0;
        if (lane == 0) q = atomicAdd(&counters[1], 1);
        q = __shfl(q, 0) + meta.n_team;
        if (q >= meta.batch) break;
        const int g = meta.order[q];
        const int64_t n = meta.ns[g], off = meta.offsets[g];
        TR(*buf)[kBatchBS] = reinterpret_cast<TR(*)[kBatchBS]>(lwave + wave * 8 * kBatchBS);
        if (wave_solve<Ar, Tin, kDual>(ar, dist, nullptr, status, g, n, off, buf, buf + 4)) continue;
        if constexpr (kDual) {
            using TA = typename Alt::T;
            TA(*abuf)[kBatchBS] = reinterpret_cast<TA(*)[kBatchBS]>(lwave + wave * 8 * kBatchBS);
            wave_solve<Alt, Tin>(alt, dist, nullptr, status, g, n, off, abuf, abuf + 4);
        }
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&counters[2], 1) == (int)gridDim.x - 1) {
            counters[0] = 0;
            counters[1] = 0;
            counters[2] = 0;
            __threadfence();
        }
    }
}

}  // namespace apsp

// --------------------------------------------------------------- plans
using namespace apsp;

struct apsp_batch_plan {
    int device = 0;
    apsp_dtype_t dtype = APSP_INT32;
    int32_t want_pred = 0;
    int32_t batch = 0;
    int32_t n_team = 0;
    int grid = 0;
    int64_t scratch_elems = 0;
    bool lean = false;         // the lean distance kernel (see batch_meta)
    int64_t max_end = 0;       // elements the packed buffers must hold
    void *dev_meta = nullptr;  // order | ns | offsets
    void *scratch = nullptr;
    int32_t *counters = nullptr;
};

namespace {

thread_local int t_last_hip = 0;

apsp_status_t plan_free(apsp_batch_plan_t *p) {
    if (!p) return APSP_SUCCESS;
    apsp_status_t st = APSP_SUCCESS;
    if (p->dev_meta && hipFree(p->dev_meta) != hipSuccess) st = APSP_ERROR_HIP;
    if (p->scratch && hipFree(p->scratch) != hipSuccess) st = APSP_ERROR_HIP;
    if (p->counters && hipFree(p->counters) != hipSuccess) st = APSP_ERROR_HIP;
    delete p;
    return st;
}

// Plans of apsp_solve_batched are freed once their stream has passed them
// (an event per plan, swept on later calls and on apsp_release_workspace).
std::mutex g_retired_mu;
std::vector<std::pair<apsp_batch_plan_t *, hipEvent_t>> g_retired;

apsp_status_t retire(apsp_batch_plan_t *p, hipStream_t s) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess) {
        (void)hipStreamSynchronize(s);  // (the plan is freed once its work is done either way)
        plan_free(p);
        return APSP_SUCCESS;
    }
    std::lock_guard<std::mutex> lk(g_retired_mu);
    g_retired.push_back({p, ev});
    return APSP_SUCCESS;
}

template <class Tin, class Ar, class Alt, int SEL = kEveryGraph>
apsp_status_t launch(const BatchLaunch &L, void *dist, int32_t *pred, int32_t *status, hipStream_t s,
                     Ar ar, Alt alt, int32_t *counters) {
    BatchMeta m;
    m.order = (const int32_t *)L.meta;
    m.ns = m.order + L.batch;
    m.offsets = (const int64_t *)((const char *)L.meta + (size_t)L.batch * 8);
    m.cfg = (const int8_t *)((const char *)L.meta + (size_t)L.batch * 16);
    m.batch = L.batch;
    m.n_team = L.n_team;
    m.scratch_elems = L.scratch_elems;
    hipLaunchKernelGGL((batched_kernel<Tin, Ar, Alt, SEL>), dim3(L.grid), dim3(kBatchThreads), 0, s, m,
                       (Tin *)dist, pred, status, L.scratch, counters, ar, alt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_last_hip = (int)e;
        return APSP_ERROR_HIP;
    }
    return APSP_SUCCESS;
}

template <class Tin, class Ar, class Alt>
apsp_status_t launch_lean(const BatchLaunch &L, void *dist, int32_t *status, hipStream_t s, Ar ar, Alt alt,
                          int32_t *counters) {
    BatchMeta m;
    m.order = (const int32_t *)L.meta;
    m.ns = m.order + L.batch;
    m.offsets = (const int64_t *)((const char *)L.meta + (size_t)L.batch * 8);
    m.cfg = (const int8_t *)((const char *)L.meta + (size_t)L.batch * 16);
    m.batch = L.batch;
    m.n_team = L.n_team;
    m.scratch_elems = L.scratch_elems;
    hipLaunchKernelGGL((batched_lean_kernel<Tin, Ar, Alt>), dim3(L.grid), dim3(kBatchThreads), 0, s, m,
                       (Tin *)dist, status, L.scratch, counters, ar, alt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_last_hip = (int)e;
        return APSP_ERROR_HIP;
    }
    return APSP_SUCCESS;
}

}  // namespace

namespace apsp {

// Workgroups of a batched launch resident on one CU (the plan's grid is
// CUs times this).
int batched_blocks_per_cu(apsp_dtype_t dtype, bool lean) {
    int blocks = 0;
    hipError_t e = hipSuccess;
    if (lean && dtype == APSP_INT32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_lean_kernel<int32_t, ArF32, ArI32>,
                                                         kBatchThreads, 0);
    else if (lean)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_lean_kernel<float, ArF32, NoAlt>,
                                                         kBatchThreads, 0);
    else
        return 2;
    return (e == hipSuccess && blocks > 0) ? blocks : 2;
}

apsp_status_t batched_launch(const BatchLaunch &L, apsp_dtype_t dtype, bool want_pred, void *dist,
                             int32_t *pred, int32_t *status, hipStream_t s) {
    if (L.batch == 0) return APSP_SUCCESS;
    if (L.lean) {  // distances; one launch with both arithmetics for int32 weights
        if (dtype == APSP_INT32)
            return launch_lean<int32_t>(L, dist, status, s, ArF32{}, ArI32{}, L.counters);
        return launch_lean<float>(L, dist, status, s, ArF32{}, NoAlt{}, L.counters);
    }
    if (dtype == APSP_INT32) {
        if (want_pred) return launch<int32_t>(L, dist, pred, status, s, ArKey{7}, NoAlt{}, L.counters);
        // int32 arithmetic for the graphs that need it, then float32 for the
        // rest; each launch has its own counters
        apsp_status_t st = launch<int32_t, ArI32, NoAlt, kIntGraphs>(L, dist, nullptr, status, s, ArI32{},
                                                                    NoAlt{}, L.counters);
        if (st != APSP_SUCCESS) return st;
        return launch<int32_t, ArF32, NoAlt, kFloatGraphs>(L, dist, nullptr, status, s, ArF32{}, NoAlt{},
                                                           L.counters + 4);
    }
    if (want_pred) return launch<float>(L, dist, pred, status, s, ArKey{7}, ArLexF32{}, L.counters);
    return launch<float>(L, dist, nullptr, status, s, ArF32{}, NoAlt{}, L.counters);
}

// ------------------------------------------------------- tuning table
// Team configuration per (dtype, predecessors, size class); size classes
// are n in (64,128], (128,192], ..., (448,512] (64 wide, so a class pads
// its graphs to one multiple of 64) and (512,1024].  Distances run in the
// lean kernel (padding to 64): 64-wide blocks up to n = 192, kMixed128
// above (measured on MI355X, 4096 graphs of one size: n = 128 0.81 vs
// 1.00 ms, 192 2.06 vs 2.23, 256 3.80 vs 3.81, 384 in 3072 graphs 10.1 vs
// 8.9); 8-byte keys keep the 64-wide configurations of the general kernel.
std::mutex g_tune_mu;
constexpr int8_t kW = kWaveTiles64, kG = kGroupTiles64, kM = kMixed128;
int8_t g_tune[2][2][kClasses] = {
    // int32: distances, predecessors
    {{kG, kG, kM, kM, kM, kM, kM, kM}, {kG, kG, kG, kW, kW, kW, kW, kW}},
    // float32
    {{kG, kG, kM, kM, kM, kM, kM, kM}, {kG, kG, kG, kW, kW, kW, kW, kW}}};
bool g_tune_env_checked = false;

apsp_status_t tune_load_locked(const char *path);

int8_t batch_config(int64_t n, apsp_dtype_t dtype, bool pred) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_env_checked) {
        g_tune_env_checked = true;
        if (const char *env = std::getenv("APSP_TUNE_TABLE")) tune_load_locked(env);
    }
    return g_tune[dtype == APSP_FLOAT32][pred ? 1 : 0][size_class(n)];
}

// JSON form of the table:
//   {"version": 2, "classes": [128, 192, 256, 320, 384, 448, 512, 1024],
//    "configs": ["wave_tiles_64", "group_tiles_64", "group_tiles_128", "mixed_128"],
//    "table": {"int32": {"dist": [c0..c7], "pred": [..]}, "float32": {...}}}
apsp_status_t tune_load_locked(const char *path) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return APSP_ERROR_INVALID_ARGUMENT;
    std::string text;
    char chunk[4096];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof chunk, f)) > 0) text.append(chunk, got);
    std::fclose(f);
    int8_t t[2][2][kClasses];
    const char *dts[2] = {"\"int32\"", "\"float32\""};
    const char *modes[2] = {"\"dist\"", "\"pred\""};
    for (int d = 0; d < 2; ++d) {
        const size_t pd = text.find(dts[d]);
        if (pd == std::string::npos) return APSP_ERROR_INVALID_VALUE;
        for (int m = 0; m < 2; ++m) {
            const size_t pm = text.find(modes[m], pd);
            const size_t lb = pm == std::string::npos ? pm : text.find('[', pm);
            if (lb == std::string::npos) return APSP_ERROR_INVALID_VALUE;
            const char *q = text.c_str() + lb + 1;
            for (int c = 0; c < kClasses; ++c) {
                char *end = nullptr;
                const long v = std::strtol(q, &end, 10);
                if (end == q || v < kWaveTiles64 || v > kMixed128) return APSP_ERROR_INVALID_VALUE;
                t[d][m][c] = (int8_t)v;
                q = end;
                while (*q == ' ' || *q == ',' || *q == '\n') ++q;
            }
        }
    }
    std::memcpy(g_tune, t, sizeof t);
    return APSP_SUCCESS;
}

apsp_status_t tune_save_locked(const char *path) {
    FILE *f = std::fopen(path, "wb");
    if (!f) return APSP_ERROR_INVALID_ARGUMENT;
    std::fprintf(f, "{\"version\": 2, \"classes\": [");
    for (int c = 0; c < kClasses; ++c) std::fprintf(f, "%s%d", c ? ", " : "", kClassHi[c]);
    std::fprintf(f, "],\n");
    std::fprintf(f, " \"configs\": [\"wave_tiles_64\", \"group_tiles_64\", \"group_tiles_128\", \"mixed_128\"],\n");
    std::fprintf(f, " \"table\": {");
    const char *dts[2] = {"int32", "float32"};
    for (int d = 0; d < 2; ++d) {
        std::fprintf(f, "%s\"%s\": {", d ? ", " : "", dts[d]);
        for (int m = 0; m < 2; ++m) {
            std::fprintf(f, "%s\"%s\": [", m ? ", " : "", m ? "pred" : "dist");
            for (int c = 0; c < kClasses; ++c) std::fprintf(f, "%s%d", c ? ", " : "", (int)g_tune[d][m][c]);
            std::fprintf(f, "]");
        }
        std::fprintf(f, "}");
    }
    std::fprintf(f, "}}\n");
    return std::fclose(f) == 0 ? APSP_SUCCESS : APSP_ERROR_INVALID_ARGUMENT;
}

// Synthetic batch for tuning: graph b (one block each) gets edges with
// probability 1/2, weights 1..1000, from an integer hash of (b, i, j).
template <class T>
__global__ void tune_fill_kernel(T *buf, const int64_t *offs, const int32_t *ns, int32_t B) {
    for (int32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const int64_t n = ns[b];
        T *g = buf + offs[b];
        for (int64_t e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int64_t i = e / n, j = e - i * n;
            uint32_t h = (uint32_t)(b * 2654435761u) ^ (uint32_t)(i * 40503u) ^ (uint32_t)(j * 2246822519u);
            h ^= h >> 15;
            h *= 2246822519u;
            h ^= h >> 13;
            T w;
            if (i == j)
                w = T(0);
            else if (h & 1)
                w = T(1 + (h >> 1) % 1000);
            else if constexpr (std::is_same_v<T, int32_t>)
                w = kInf32;
            else
                w = __builtin_inff();
            g[e] = w;
        }
    }
}

// Device metadata image of a batch (see batch_meta_with) with the tuning
// table's configurations.
void batch_meta(const int32_t *ns, const int64_t *offsets, int32_t B, apsp_dtype_t dtype, bool pred,
                const int8_t *forced, std::vector<char> &bytes, int32_t &n_team, int64_t &scratch_elems,
                bool &lean) {
    batch_meta_with(ns, offsets, B, pred, forced, [&](int64_t n) { return batch_config(n, dtype, pred); }, bytes,
                    n_team, scratch_elems, lean);
}

// wait == true: block until every retired plan can be freed.
void sweep_retired(bool wait) {
    std::lock_guard<std::mutex> lk(g_retired_mu);
    for (auto it = g_retired.begin(); it != g_retired.end();) {
        if (wait) (void)hipEventSynchronize(it->second);
        if (hipEventQuery(it->second) == hipSuccess) {
            (void)hipEventDestroy(it->second);
            plan_free(it->first);
            it = g_retired.erase(it);
        } else {
            ++it;
        }
    }
}
}  // namespace apsp

extern "C" {

apsp_status_t apsp_batch_plan_create_ex(const int32_t *ns, const int64_t *offsets, int32_t batch,
                                        apsp_dtype_t dtype, int32_t want_pred, const int8_t *team_config,
                                        apsp_batch_plan_t **out_plan) {
    if (!out_plan) return APSP_ERROR_INVALID_ARGUMENT;
    sweep_retired(false);
    *out_plan = nullptr;
    if (dtype != APSP_INT32 && dtype != APSP_FLOAT32) return APSP_ERROR_INVALID_ARGUMENT;
    int64_t max_end = 0;
    const apsp_status_t bad = plan_args_check(ns, offsets, batch, team_config, &max_end);
    if (bad != APSP_SUCCESS) return bad;

    auto *p = new (std::nothrow) apsp_batch_plan_t();
    if (!p) return APSP_ERROR_OUT_OF_MEMORY;
    p->dtype = dtype;
    p->want_pred = want_pred ? 1 : 0;
    p->batch = batch;
    p->max_end = max_end;
    if (hipGetDevice(&p->device) != hipSuccess) {
        plan_free(p);
        return APSP_ERROR_HIP;
    }
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) cus = 256;
    std::vector<char> host;
    batch_meta(ns, offsets, batch, dtype, p->want_pred, team_config, host, p->n_team, p->scratch_elems, p->lean);
    p->grid = std::max(1, batched_blocks_per_cu(dtype, p->lean) * cus);
    const size_t elem = p->want_pred ? 8 : 4;
    if (hipMalloc(&p->dev_meta, host.size()) != hipSuccess ||
        hipMalloc((void **)&p->counters, 8 * sizeof(int32_t)) != hipSuccess ||
        (p->scratch_elems > 0 &&
         hipMalloc(&p->scratch, (size_t)p->grid * p->scratch_elems * elem) != hipSuccess)) {
        plan_free(p);
        return APSP_ERROR_OUT_OF_MEMORY;
    }
    // (the memset is on the null stream: wait for it, so a launch on a
    // non-blocking stream cannot overtake it)
    if (hipMemcpy(p->dev_meta, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(p->counters, 0, 8 * sizeof(int32_t)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        plan_free(p);
        return APSP_ERROR_HIP;
    }
    *out_plan = p;
    return APSP_SUCCESS;
}

apsp_status_t apsp_batch_plan_create(const int32_t *ns, const int64_t *offsets, int32_t batch,
                                     apsp_dtype_t dtype, int32_t want_pred, apsp_batch_plan_t **out_plan) {
    return apsp_batch_plan_create_ex(ns, offsets, batch, dtype, want_pred, nullptr, out_plan);
}

apsp_status_t apsp_batch_plan_execute(const apsp_batch_plan_t *plan, void *packed_dist,
                                      int32_t *packed_pred, int32_t *d_status, hipStream_t stream) {
    if (!plan) return APSP_ERROR_INVALID_ARGUMENT;
    if (plan->batch == 0) return APSP_SUCCESS;
    if (!packed_dist || (plan->want_pred && !packed_pred) || (!plan->want_pred && packed_pred))
        return APSP_ERROR_INVALID_ARGUMENT;
    if ((uintptr_t)packed_dist % 16 || (uintptr_t)packed_pred % 16) return APSP_ERROR_INVALID_ARGUMENT;
    BatchLaunch L{plan->dev_meta, plan->batch, plan->n_team, plan->scratch_elems, plan->scratch,
                  plan->counters, plan->grid, plan->lean};
    return batched_launch(L, plan->dtype, plan->want_pred, packed_dist, packed_pred, d_status, stream);
}

apsp_status_t apsp_batch_plan_destroy(apsp_batch_plan_t *plan) { return plan_free(plan); }

int32_t apsp_batch_config(int64_t n, apsp_dtype_t dtype, int32_t want_pred) {
    if (n <= kBatchBS) return -1;  // solved by one wavefront in registers
    return batch_config(n, dtype, want_pred != 0);
}

apsp_status_t apsp_tune_load(const char *path) {
    if (!path) return APSP_ERROR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_env_checked = true;
    return tune_load_locked(path);
}

apsp_status_t apsp_tune_save(const char *path) {
    if (!path) return APSP_ERROR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return tune_save_locked(path);
}

}  // extern "C"

namespace {

// Coordinate descent over the size classes present in `sizes` (graphs of
// those sizes, synthetic weights): one class at a time, the others at
// their current choice, the whole batch timed for each configuration.
apsp_status_t autotune_on(const std::vector<int32_t> &sizes, apsp_dtype_t dtype, int32_t want_pred, int32_t reps,
                          double *ms_out) {
    const int R = reps ? reps : 3;
    const int d = dtype == APSP_FLOAT32, m = want_pred ? 1 : 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune_env_checked) {
            g_tune_env_checked = true;
            if (const char *env = std::getenv("APSP_TUNE_TABLE")) tune_load_locked(env);
        }
    }
    const int32_t B = (int32_t)sizes.size();
    std::vector<int32_t> ns(sizes), cls(B);
    std::vector<int64_t> offs(B);
    bool present[kClasses] = {};
    int64_t total = 0;
    for (int32_t b = 0; b < B; ++b) {
        cls[b] = ns[b] <= kBatchBS ? -1 : size_class(ns[b]);  // n <= 64: one wavefront, no team
        if (cls[b] >= 0) present[cls[b]] = true;
        offs[b] = total;
        total += ((int64_t)ns[b] * ns[b] + 3) / 4 * 4;
    }
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return APSP_ERROR_HIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *dist = nullptr, *pred = nullptr, *meta = nullptr;
    apsp_status_t result = APSP_SUCCESS;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) result = APSP_ERROR_HIP;
    if (result == APSP_SUCCESS &&
        (hipMalloc(&dist, (size_t)total * 4) != hipSuccess ||
         (want_pred && hipMalloc(&pred, (size_t)total * 4) != hipSuccess) ||
         hipMalloc(&meta, (size_t)B * 12) != hipSuccess))
        result = APSP_ERROR_OUT_OF_MEMORY;
    if (result == APSP_SUCCESS &&
        (hipMemcpy(meta, offs.data(), (size_t)B * 8, hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy((char *)meta + (size_t)B * 8, ns.data(), (size_t)B * 4, hipMemcpyHostToDevice) != hipSuccess))
        result = APSP_ERROR_HIP;
    if (result == APSP_SUCCESS) {
        const int32_t *dns = (const int32_t *)((char *)meta + (size_t)B * 8);
        if (dtype == APSP_INT32)
            hipLaunchKernelGGL(tune_fill_kernel<int32_t>, dim3(std::min(B, 4096)), dim3(256), 0, s,
                               (int32_t *)dist, (const int64_t *)meta, dns, B);
        else
            hipLaunchKernelGGL(tune_fill_kernel<float>, dim3(std::min(B, 4096)), dim3(256), 0, s,
                               (float *)dist, (const int64_t *)meta, dns, B);
    }
    int8_t choice[kClasses];
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        std::memcpy(choice, g_tune[d][m], sizeof choice);
    }
    auto time_batch = [&](const int8_t *ch, double &ms_per) -> apsp_status_t {
        std::vector<int8_t> forced(B);
        for (int32_t b = 0; b < B; ++b) forced[b] = cls[b] >= 0 ? ch[cls[b]] : (int8_t)-1;
        apsp_batch_plan_t *plan = nullptr;
        apsp_status_t st =
            apsp_batch_plan_create_ex(ns.data(), offs.data(), B, dtype, want_pred, forced.data(), &plan);
        if (st != APSP_SUCCESS) return st;
        st = apsp_batch_plan_execute(plan, dist, (int32_t *)pred, nullptr, s);  // warm-up
        if (st == APSP_SUCCESS && hipEventRecord(e0, s) != hipSuccess) st = APSP_ERROR_HIP;
        for (int r = 0; r < R && st == APSP_SUCCESS; ++r)
            st = apsp_batch_plan_execute(plan, dist, (int32_t *)pred, nullptr, s);
        float ms = 0.f;
        if (st == APSP_SUCCESS &&
            (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = APSP_ERROR_HIP;
        plan_free(plan);
        ms_per = (double)ms / R;
        return st;
    };
    // coordinate descent: one class at a time, the others at their current choice
    for (int c = 0; c < kClasses && result == APSP_SUCCESS; ++c) {
        if (!present[c]) continue;
        double best_ms = 1e300;
        int best = choice[c];
        // the mixed configuration is a distance configuration (the lean kernel)
        const int last = want_pred ? kGroupTiles128 : kMixed128;
        for (int cfg = kWaveTiles64; cfg <= last && result == APSP_SUCCESS; ++cfg) {
            int8_t trial[kClasses];
            std::memcpy(trial, choice, sizeof trial);
            trial[c] = (int8_t)cfg;
            double ms = 0.0;
            result = time_batch(trial, ms);
            if (ms_out) ms_out[c * 4 + cfg] = ms;
            if (result == APSP_SUCCESS && ms < best_ms) {
                best_ms = ms;
                best = cfg;
            }
        }
        choice[c] = (int8_t)best;
    }
    if (result == APSP_SUCCESS) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        std::memcpy(g_tune[d][m], choice, sizeof choice);
    }
    if (hipStreamSynchronize(s) != hipSuccess && result == APSP_SUCCESS) result = APSP_ERROR_HIP;
    (void)hipFree(dist);
    (void)hipFree(pred);
    (void)hipFree(meta);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return result;
}

}  // namespace

extern "C" {

apsp_status_t apsp_batch_autotune(apsp_dtype_t dtype, int32_t want_pred, int32_t graphs_per_class,
                                  int32_t reps, double *ms_out) {
    if (dtype != APSP_INT32 && dtype != APSP_FLOAT32) return APSP_ERROR_INVALID_ARGUMENT;
    if (graphs_per_class < 0 || reps < 0) return APSP_ERROR_INVALID_ARGUMENT;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess) return APSP_ERROR_HIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    const int32_t per = graphs_per_class ? graphs_per_class : cus;
    // `per` graphs spread evenly over every size class
    std::vector<int32_t> sizes;
    for (int c = 0; c < kClasses; ++c) {
        const int lo = c == 0 ? kBatchBS + 1 : kClassHi[c - 1] + 1, hi = kClassHi[c];
        for (int32_t q = 0; q < per; ++q) sizes.push_back(lo + (int32_t)(((int64_t)q * (hi - lo + 1)) / per));
    }
    return autotune_on(sizes, dtype, want_pred, reps, ms_out);
}

apsp_status_t apsp_batch_autotune_sizes(const int32_t *ns, int32_t batch, apsp_dtype_t dtype, int32_t want_pred,
                                        int32_t reps, double *ms_out) {
    if (dtype != APSP_INT32 && dtype != APSP_FLOAT32) return APSP_ERROR_INVALID_ARGUMENT;
    if (!ns || batch <= 0 || reps < 0) return APSP_ERROR_INVALID_ARGUMENT;
    std::vector<int32_t> sizes(ns, ns + batch);
    for (int32_t v : sizes)
        if (v < 1 || v > kClassHi[kClasses - 1]) return APSP_ERROR_INVALID_ARGUMENT;
    return autotune_on(sizes, dtype, want_pred, reps, ms_out);
}

apsp_status_t apsp_solve_batched(void *packed_dist, int32_t *packed_pred, const int32_t *ns,
                                 const int64_t *offsets, int32_t batch, apsp_dtype_t dtype,
                                 hipStream_t stream) {
    sweep_retired(false);
    apsp_batch_plan_t *plan = nullptr;
    apsp_status_t st =
        apsp_batch_plan_create(ns, offsets, batch, dtype, packed_pred != nullptr ? 1 : 0, &plan);
    if (st != APSP_SUCCESS) return st;
    st = apsp_batch_plan_execute(plan, packed_dist, packed_pred, nullptr, stream);
    if (st != APSP_SUCCESS) {
        plan_free(plan);
        return st;
    }
    return retire(plan, stream);
}

}  // extern "C"
