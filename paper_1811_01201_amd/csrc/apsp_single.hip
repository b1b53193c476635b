// Single-graph blocked Floyd–Warshall for gfx950.
//
// The round structure follows the paper's Section "Data Locality": for each
// k-block r the diagonal block is closed first (phase 1), then the rest of
// block row r and block column r (phase 2), then every other block from its
// row's and column's panel blocks (phase 3).  Phase 2 is written here as a
// min-plus product against the closed diagonal block (a path from the block
// row to any vertex leaves block r for the last time at some k in block r),
// which gives the same values as the paper's in-place sweep and lets all
// three phases share one register-blocked tile routine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <tuple>
#include <type_traits>
#include <map>
#include <mutex>
#include <vector>

#include "apsp_internal.h"

// Launch tuning (measured on MI355X): phase-3 waves per SIMD for 4-byte
// elements on 128 x 128 tiles (157 VGPRs) and for 8-byte keys; phase-2
// waves per SIMD for 4-byte elements (at most 168 VGPRs, so a phase-2
// workgroup fits on a compute unit beside two phase-3 workgroups and starts
// while a remaining-block launch runs: at n = 16384 the next round's panels
// then finish mid-launch instead of 33 us after it, 110.3 vs 110.6 ms; at
// 32768 848.2 vs 851.6 ms); kRest launches per round under the two-stream
// schedule.
constexpr int kP3Waves4 = 3;
constexpr int kP3Waves8 = 2;
constexpr int kP2Waves4 = 3;
constexpr int kRestChunks = 2;

namespace apsp {

template <class Ar, class Alt, int BS, int TT>
__global__ void __launch_bounds__((P1S<Ar, BS, TT>::NTH))
__attribute__((amdgpu_waves_per_eu(P1S<Ar, BS, TT>::kWavesPerSimd, P1S<Ar, BS, TT>::kWavesPerSimd)))
phase1_kernel(void *X, int64_t ld, int64_t r0, Ar ar, Alt alt, const int32_t *__restrict__ mode,
              const int32_t *__restrict__ skip) {
    static_assert(std::is_same_v<Alt, NoAlt> || P1S<Ar, BS, TT>::NTH == P1S<Alt, BS, TT>::NTH,
                  "both policies close the block with the same workgroup");
    if (skip && *skip != APSP_SUCCESS) return;
    constexpr int E = sizeof(typename Ar::T) > sizeof(typename Alt::T) ? sizeof(typename Ar::T)
                                                                        : sizeof(typename Alt::T);
    __shared__ __attribute__((aligned(16))) char lds[2 * 4 * BS * E];  // 4 column + 4 row buffers
    if constexpr (!std::is_same_v<Alt, NoAlt>) {
        if (use_alt<Ar, Alt>(mode)) {
            using T = typename Alt::T;
            phase1_body<Alt, BS, false, TT>((T *)X, ld, r0, alt, (T(*)[BS])lds,
                                            (T(*)[BS])(lds + 4 * BS * sizeof(T)));
            return;
        }
    }
    using T = typename Ar::T;
    phase1_body<Ar, BS, false, TT>((T *)X, ld, r0, ar, (T(*)[BS])lds, (T(*)[BS])(lds + 4 * BS * sizeof(T)));
}

// Phase 1 at BS = 256 for 4-byte elements without a second policy: the
// diagonal block closed by a blocked Floyd-Warshall of its own inside one
// 256-thread workgroup, four 64-wide rounds of (64 x 64 diagonal closure;
// its block row and column as products against it; the other nine 64 x 64
// tiles as products), which reaches the values of 256 single steps by the
// blocked schedule's own argument.  Every product is watched (inputs and
// outputs) as well as every closure's publications and results, so a
// watching policy still sees each operand.  Its registers and LDS fit in
// what one phase-3 workgroup frees: it starts as soon as any of those
// finishes, where the one-step-per-barrier kernel needs a whole compute
// unit to drain.
template <class Ar>
__global__ void __launch_bounds__(256) phase1_blocked_kernel(void *X, int64_t ld, int64_t r0, Ar ar,
                                                             const int32_t *__restrict__ skip) {
    using T = typename Ar::T;
    using GT = TileProductDMA<Ar, 64, 64, 16, 4, 4>;
    static_assert(sizeof(T) == 4 && GT::NTH == 256 && P1S<Ar, 64, 4>::NTH == 256, "one 256-thread workgroup");
    if (skip && *skip != APSP_SUCCESS) return;
    __shared__ union alignas(16) {
        typename GT::Smem t;
        T p1[8 * 64];  // closure publications: 4 column + 4 row buffers
    } sm;
    T *const D = (T *)X;
    T(*const buf)[64] = reinterpret_cast<T(*)[64]>(sm.p1);
    for (int s = 0; s < 4; ++s) {
        const int64_t d0 = r0 + 64 * s;
        phase1_body<Ar, 64, false, 4>(D, ld, d0, ar, buf, buf + 4);
        __syncthreads();
        for (int t = 0; t < 6; ++t) {  // block row s (t < 3) and block column s
            int q = t % 3;
            q += (q >= s) ? 1 : 0;
            const int64_t o = r0 + 64 * q;
            if (t < 3)
                GT::template run<true>(sm.t, D, ld, d0, o, d0, 64, ar);
            else
                GT::template run<true>(sm.t, D, ld, o, d0, d0, 64, ar);
        }
        __syncthreads();
        for (int t = 0; t < 9; ++t) {
            int a = t / 3, b = t % 3;
            a += (a >= s) ? 1 : 0;
            b += (b >= s) ? 1 : 0;
            GT::template run<true>(sm.t, D, ld, r0 + 64 * a, r0 + 64 * b, d0, 64, ar);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- phase 2
// Block row r:    C = D[r-block rows, J cols] (BS x P2W tiles), A = closed
//                 diagonal block, B = C's own old values.
// Block column r: C = D[I rows, r-block cols] (P2W x BS tiles), A = C's own
//                 old values, B = closed diagonal block.
// Each tile spans the whole k-block along the direction it reads from
// itself, so it can update in place.  Workgroups [0, nt) do the row panel,
// [nt, 2 nt) the column panel; nt = number of P2W-wide tiles outside block r.
template <class Ar, int BS, int P2W, int TT>
struct P2 {
    // 4-byte elements: LDS DMA; 8-byte keys strip A while staging it instead
    using RowT = std::conditional_t<sizeof(typename Ar::T) == 4, TileProductDMA<Ar, BS, P2W, 16, TT, TT>,
                                    TileProduct<Ar, BS, P2W, 16, TT, TT>>;
    using ColT = std::conditional_t<sizeof(typename Ar::T) == 4, TileProductDMA<Ar, P2W, BS, 16, TT, TT>,
                                    TileProduct<Ar, P2W, BS, 16, TT, TT>>;
    static_assert(RowT::NTH == ColT::NTH, "both panel shapes use one block size");
    union Smem {
        typename RowT::Smem row;
        typename ColT::Smem col;
    };
    __device__ __forceinline__ static void run(Smem &sm, typename Ar::T *D, int64_t ld, int64_t r0,
                                               int nt, const Ar &ar) {
        int t = blockIdx.x;
        const bool is_row = t < nt;
        if (!is_row) t -= nt;
        const int per_block = BS / P2W;
        const int rb = (int)(r0 / P2W);
        const int tt = t + (t >= rb ? per_block : 0);  // skip the diagonal block's tiles
        const int64_t off = (int64_t)tt * P2W;
        // the panels are phase 3's operands: a watching policy checks them
        if (is_row)
            RowT::template run<Ar::kWatch>(sm.row, D, ld, r0, off, r0, BS, ar);
        else
            ColT::template run<Ar::kWatch>(sm.col, D, ld, off, r0, r0, BS, ar);
    }
};

template <class T>
constexpr int elem_size() {
    return sizeof(T);
}
template <>
constexpr int elem_size<char>() {
    return 0;
}

template <class Ar, class Alt, int BS, int P2W, int TT>
__global__ void __launch_bounds__((BS / TT) * (P2W / TT))
__attribute__((amdgpu_waves_per_eu(sizeof(typename Ar::T) == 4 ? kP2Waves4 : 1)))
phase2_kernel(void *X, int64_t ld, int64_t r0, int nt, Ar ar, Alt alt,
              const int32_t *__restrict__ mode, const int32_t *__restrict__ skip) {
    if (skip && *skip != APSP_SUCCESS) return;
    if constexpr (!std::is_same_v<Alt, NoAlt>) {
        __shared__ union {
            typename P2<Ar, BS, P2W, TT>::Smem a;
            typename P2<Alt, BS, P2W, TT>::Smem b;
        } sm;
        if (use_alt<Ar, Alt>(mode))
            P2<Alt, BS, P2W, TT>::run(sm.b, (typename Alt::T *)X, ld, r0, nt, alt);
        else
            P2<Ar, BS, P2W, TT>::run(sm.a, (typename Ar::T *)X, ld, r0, nt, ar);
    } else {
        __shared__ typename P2<Ar, BS, P2W, TT>::Smem sm;
        P2<Ar, BS, P2W, TT>::run(sm, (typename Ar::T *)X, ld, r0, nt, ar);
    }
}

// ---------------------------------------------------------------- phase 3
// Every tile outside block row r and block column r:
//     C <- min(C, D[C rows, r-block] (x) D[r-block, C cols]).
// Workgroup ids are remapped so that each of the 8 XCDs (a dispatch places
// workgroup w on XCD w mod 8) walks its own contiguous stretch of a grouped
// tile order: GROUP tile rows at a time, all columns, so the panel slices
// that the XCD's resident workgroups read stay in that XCD's L2.
// Tile sets of phase 3 (tile = MT x MT, pb = BS / MT tiles per block):
//   kAll    every tile outside block row r and block column r
//   kRest   every tile outside block rows/columns r and r + 1
//   kCross  the tiles of block row r + 1 and block column r + 1 outside
//           block row/column r (the next round's diagonal and panels)
// kRest + kCross = kAll.  The two-stream schedule runs kCross on the
// critical path and kRest beside the next round's phases 1 and 2.
enum P3Set { kAll = 0, kRest = 1, kCross = 2 };

__host__ __device__ inline int64_t p3_count(int set, int nt, int pb) {
    if (set == kAll) return (int64_t)(nt - pb) * (nt - pb);
    if (set == kRest) return (int64_t)(nt - 2 * pb) * (nt - 2 * pb);
    return (int64_t)pb * (nt - pb) + (int64_t)(nt - 2 * pb) * pb;
}

// Maps workgroup blockIdx.x to a tile; false if it has none.  kAll/kRest
// walk a grouped order (GROUP tile rows at a time, all columns), each of the
// 8 XCDs (a dispatch places workgroup w on XCD w mod 8) taking its own
// contiguous stretch so the panel slices its resident workgroups read stay
// in that XCD's L2.
__device__ __forceinline__ bool phase3_tile(int set, int r, int nt, int pb, int per_xcd, int seq0,
                                            int seq_end, int MT, int64_t &crow, int64_t &ccol) {
    constexpr int GROUP = 8;
    const int w = blockIdx.x;
    const int seq = seq0 + (w & 7) * per_xcd + (w >> 3);
    if (seq >= seq_end) return false;
    const int e1 = r * pb;  // first tile index of block r
    int ti, tj;
    if (set == kCross) {
        const int nrow = pb * (nt - pb);
        if (seq < nrow) {  // rows of block r + 1, columns outside block r
            ti = (r + 1) * pb + seq / (nt - pb);
            tj = seq % (nt - pb);
            tj += (tj >= e1) ? pb : 0;
        } else {           // columns of block r + 1, rows outside blocks r, r + 1
            const int q = seq - nrow;
            ti = q / pb;
            tj = (r + 1) * pb + q % pb;
            ti += (ti >= e1) ? 2 * pb : 0;
        }
    } else {
        const int skip = (set == kAll) ? pb : 2 * pb;  // excluded tiles start at e1
        const int ntr = nt - skip;
        const int group = seq / (GROUP * ntr);
        const int first = group * GROUP;
        const int rows = min(GROUP, ntr - first);
        const int within = seq - group * GROUP * ntr;
        ti = first + within % rows;
        tj = within / rows;
        ti += (ti >= e1) ? skip : 0;
        tj += (tj >= e1) ? skip : 0;
    }
    crow = (int64_t)ti * MT;
    ccol = (int64_t)tj * MT;
    return true;
}

template <class Ar, class Alt, int BS, int MT, int SET, int TT>
__global__ void __launch_bounds__((MT / TT) * (MT / TT))
__attribute__((amdgpu_waves_per_eu(sizeof(typename Ar::T) == 4 ? (MT == 128 ? kP3Waves4 : 2) : kP3Waves8)))
phase3_kernel(void *X, int64_t ld, int r, int per_xcd, int seq0, int seq_end, Ar ar, Alt alt,
              const int32_t *__restrict__ mode, const int32_t *__restrict__ skip) {
    constexpr int set = SET;
    // LDS DMA staging (8-byte keys: stripped in LDS after each chunk arrives)
    using TP = TileProductDMA<Ar, MT, MT, 16, TT, TT>;
    if (skip && *skip != APSP_SUCCESS) return;
    int64_t crow, ccol;
    if (!phase3_tile(set, r, (int)(ld / MT), BS / MT, per_xcd, seq0, seq_end, MT, crow, ccol)) return;
    const int64_t r0 = (int64_t)r * BS;
    if constexpr (!std::is_same_v<Alt, NoAlt>) {
        using TQ = std::conditional_t<sizeof(typename Alt::T) == 4, TileProductDMA<Alt, MT, MT, 16, TT, TT>,
                                      TileProduct<Alt, MT, MT, 16, TT, TT>>;
        __shared__ union {
            typename TP::Smem a;
            typename TQ::Smem b;
        } sm;
        if (use_alt<Ar, Alt>(mode))
            TQ::run(sm.b, (typename Alt::T *)X, ld, crow, ccol, r0, BS, alt);
        else
            TP::run(sm.a, (typename Ar::T *)X, ld, crow, ccol, r0, BS, ar);
    } else {
        __shared__ typename TP::Smem sm;
        TP::run(sm, (typename Ar::T *)X, ld, crow, ccol, r0, BS, ar);
    }
}

// --------------------------------------------- dataflow (task graph) solves
// Below n of a few thousand a solve is a chain of dependent launches whose
// dispatch gaps, not their arithmetic, set the time; and phase 1 of 128-
// and 256-wide blocks is a chain of dependent steps on one compute unit.
// Both are served by one kernel (flow_tasks_kernel below) that runs the
// blocked schedule over small blocks as a graph of tasks inside a single
// launch.
//
// Coherence without cache flushes: each XCD has its own L2, and a
// device-scope release or acquire fence writes back or invalidates the
// whole L2 (measured on MI355X: one per wavefront made a 1024-workgroup
// barrier cost 62 us).  Instead every load and store of the matrix in these
// kernels is device-coherent (cache policy sc1: stores write through, loads
// do not return lines another XCD may have overwritten), so a task only
// waits for its own stores to complete before it marks its result ready.
constexpr int kSingleBS = 64;         // the solve's block size the single launch belongs to
constexpr int kSingleThreads = 256;
// element offsets within the matrix are 32-bit
constexpr int64_t kSingleMaxN = 16384;
// Polls of one wait before it gives up (about a second or more; every wait
// is for a task that running workgroups hold, so it ends long before unless
// the device is broken).  A failed wait sets the fail word, which ends
// every other wait, and the solve reports APSP_ERROR_TIMEOUT.
constexpr uint32_t kBarrierSpins = 1u << 22;

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// this wavefront's loads and stores (device-coherent ones included) complete
__device__ __forceinline__ void mem_done() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// 16-byte device-coherent accesses (two 8-byte device-scope atomics, which
// the compiler emits as dwordx2 loads and stores with sc1)
template <class T>
__device__ __forceinline__ void ld16_dev(const T *p, T *out) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    const uint64_t *q = (const uint64_t *)p;
    const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    out[0] = __builtin_bit_cast(T, (uint32_t)a);
    out[1] = __builtin_bit_cast(T, (uint32_t)(a >> 32));
    out[2] = __builtin_bit_cast(T, (uint32_t)b);
    out[3] = __builtin_bit_cast(T, (uint32_t)(b >> 32));
}
template <class T>
__device__ __forceinline__ void st16_dev(T *p, const T *in) {
    uint64_t *q = (uint64_t *)p;
    const uint64_t a = (uint64_t)__builtin_bit_cast(uint32_t, in[0]) |
                       ((uint64_t)__builtin_bit_cast(uint32_t, in[1]) << 32);
    const uint64_t b = (uint64_t)__builtin_bit_cast(uint32_t, in[2]) |
                       ((uint64_t)__builtin_bit_cast(uint32_t, in[3]) << 32);
    __hip_atomic_store(q, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 256 threads per block: BS = 64 with 4 x 4 elements per thread, BS = 32
// with 2 x 2.
template <int BS>
constexpr int flow_tile() {
    return BS == 32 ? 2 : 4;
}

// TT consecutive 4-byte elements: plain and device-coherent accesses
template <int TT, class T>
__device__ __forceinline__ void ld_tt(const T *p, T *out) {
    if constexpr (TT == 4) {
        ld16(p, out);
    } else {
        const uint64_t v = *(const uint64_t *)p;
        out[0] = __builtin_bit_cast(T, (uint32_t)v);
        out[1] = __builtin_bit_cast(T, (uint32_t)(v >> 32));
    }
}
template <int TT, class T>
__device__ __forceinline__ void st_tt(T *p, const T *in) {
    if constexpr (TT == 4) {
        st16(p, in);
    } else {
        *(uint64_t *)p = (uint64_t)__builtin_bit_cast(uint32_t, in[0]) |
                         ((uint64_t)__builtin_bit_cast(uint32_t, in[1]) << 32);
    }
}
template <int TT, class T>
__device__ __forceinline__ void st_tt_dev(T *p, const T *in) {
    if constexpr (TT == 4) {
        st16_dev(p, in);
    } else {
        const uint64_t v = (uint64_t)__builtin_bit_cast(uint32_t, in[0]) |
                           ((uint64_t)__builtin_bit_cast(uint32_t, in[1]) << 32);
        __hip_atomic_store((uint64_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// LDS layouts of a BS x BS product's operands: A as BS rows of BS k, its
// 16-byte pieces XOR-swizzled per row (flow_swz) so the rows a wavefront
// reads at one k spread over the banks; B as BS k-rows of BS columns.
template <int BS>
__device__ __forceinline__ int flow_swz(int row) {
    constexpr int KP = BS / 4;
    return ((row * KP) >> 3) & (KP - 1);
}

// Device-coherent LDS DMA of one BS x BS block (row stride ld) into LDS as
// the A (swizzled) or B (plain) operand: 16 bytes per lane and copy.
template <int BS, int NTH, bool SWIZZLE, class T>
__device__ __forceinline__ void flow_copy(T *__restrict__ lds, const T *__restrict__ src, uint32_t ld) {
    constexpr int KP = BS / 4, COPIES = BS * KP / NTH;
    static_assert(COPIES * NTH == BS * KP, "whole copies");
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
#pragma unroll
    for (int q = 0; q < COPIES; ++q) {
        const int base = q * NTH + wave * 64, v = base + lane;
        const int row = v / KP, piece = v % KP;
        const T *g = src + ((uint32_t)row * ld + (uint32_t)((SWIZZLE ? piece ^ flow_swz<BS>(row) : piece) * 4));
        __builtin_amdgcn_global_load_lds((const void *)g, (__attribute__((address_space(3))) void *)(lds + base * 4),
                                         16, 0, kCpolDevice);
    }
}

__global__ void flow_init_kernel(uint32_t *words, int count, int32_t *status) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) words[i] = 0;
    if (status && blockIdx.x == 0 && threadIdx.x == 0) *status = APSP_SUCCESS;
}

// Dataflow solve as a ticketed task graph: the tasks of the blocked
// schedule over BS-wide blocks are numbered in an order where every task's
// operands come from tasks with smaller numbers (task_decode) --
//   0                         phase 1 of round 0 on block (0, 0)
//   then per round r:         2m panel products (block row r, then block
//                             column r; m = R - 1), then the m^2 remaining
//                             blocks: block (r+1, r+1) first (phase 3, then
//                             at once its phase 1 of round r+1), then the
//                             other blocks of block row and column r+1 (the
//                             next round's panels), then the rest
// -- and a workgroup takes the next number from a counter, waits for the
// operands it reads and does the task, over and over.  The next round's
// chain (its panels, its diagonal block) comes first in each round.  A
// task only waits for smaller numbers, which running workgroups hold, so the launch makes
// progress however few of its workgroups are resident and whatever else
// runs on the device.  Block states live in X (device-coherent loads and
// stores); panels and closed diagonal blocks are also published once each
// to P_row / P_col, so a reader never sees a later round's value.
// words: ver(i, j) at i R + j = rounds applied to block (i, j) (its panel
// or closed block is published once ver passes that round), then the fail
// word, the task counter and the finished-workgroup count; zero before a
// launch, zeroed again by the last workgroup to finish.
// (the fail word, the counter and the count 1 KiB apart: every waiting
// workgroup reads the fail word, every task bumps the counter)
__host__ __device__ constexpr int task_fail_word(int R) { return R * R + 256; }
__host__ __device__ constexpr int task_next_word(int R) { return R * R + 512; }
__host__ __device__ constexpr int task_done_word(int R) { return R * R + 768; }
__host__ __device__ constexpr int task_words(int R) { return R * R + 1024; }
__host__ __device__ constexpr size_t task_word_bytes(int R) { return (size_t)task_words(R) * 4; }
// numbers per round: m (m + 2), m = R - 1 (every round: 2m panels, m^2
// remaining blocks); in all 1 + R m (m + 2)
__host__ __device__ constexpr int64_t task_round(int R) { return (int64_t)(R - 1) * (R + 1); }
__host__ __device__ constexpr int64_t task_count(int R) { return 1 + (int64_t)R * task_round(R); }

// The task with number t: kind 0 the closure of block (0, 0); 1 the
// block-row panel (r, j); 2 the block-column panel (i, r); 3 the product of
// remaining block (i, j) in round r (block (r+1, r+1) closes itself after).
// Within round r < R - 1 the remaining blocks come as (r+1, r+1), then the
// rest of block row and column r+1, then all others (row-major); in the
// last round row-major.
struct FlowTask {
    int kind, r, i, j;
};
__device__ __forceinline__ FlowTask task_decode(uint32_t t, int R) {
    FlowTask k{0, 0, 0, 0};
    if (t == 0) return k;
    const int m = R - 1;
    const uint32_t t1 = t - 1, per = (uint32_t)task_round(R);
    k.r = (int)(t1 / per);
    int u = (int)(t1 - (uint32_t)k.r * per);
    const int r = k.r;
    if (u < 2 * m) {
        const bool row = u < m;
        int q = row ? u : u - m;
        q += q >= r;
        k.kind = row ? 1 : 2;
        k.i = row ? r : q;
        k.j = row ? q : r;
        return k;
    }
    u -= 2 * m;
    k.kind = 3;
    if (r + 1 < R) {
        const int w = m - 1;  // indices outside {r, r+1}: q -> q + (q >= r ? 2 : 0)
        if (u == 0) {
            k.i = k.j = r + 1;
        } else if (u - 1 < 2 * w) {
            const int q = (u - 1) % w, x = q + (q >= r ? 2 : 0);
            k.i = u - 1 < w ? r + 1 : x;
            k.j = u - 1 < w ? x : r + 1;
        } else {
            const int a = u - 1 - 2 * w, qi = a / w, qj = a - (a / w) * w;
            k.i = qi + (qi >= r ? 2 : 0);
            k.j = qj + (qj >= r ? 2 : 0);
        }
    } else {
        const int qi = u / m, qj = u - (u / m) * m;
        k.i = qi + (qi >= r);
        k.j = qj + (qj >= r);
    }
    return k;
}

// Waits (thread 0 polling) until *w0 >= v0 and, if w1, *w1 >= v1; the
// workgroup leaves together.  False if the wait ran out or another did.
__device__ __forceinline__ bool task_wait(const uint32_t *w0, uint32_t v0, const uint32_t *w1, uint32_t v1,
                                          uint32_t *fail, int *ok_lds) {
    if (threadIdx.x == 0) {
        int ok = 1;
        for (uint32_t spin = 0; ld_agent(w0) < v0 || (w1 && ld_agent(w1) < v1); ++spin) {
            if (spin >= kBarrierSpins) {
                st_agent(fail, 1u);
                ok = 0;
                break;
            }
            if ((spin & 31) == 31 && ld_agent(fail) != 0) {  // (now and then: one word all waiters share)
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

template <int TT, class T>
__device__ __forceinline__ void ld_tt_dev(const T *p, T *out) {
    if constexpr (TT == 4) {
        ld16_dev(p, out);
    } else {
        const uint64_t v = __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        out[0] = __builtin_bit_cast(T, (uint32_t)v);
        out[1] = __builtin_bit_cast(T, (uint32_t)(v >> 32));
    }
}

template <class Ar, int BS>
__global__ void __launch_bounds__(kSingleThreads) __attribute__((amdgpu_waves_per_eu(4)))
flow_tasks_kernel(void *Xv, int64_t order, int64_t stride, Ar ar, uint32_t *words, void *prow_v, void *pcol_v,
                  int32_t *status, const int32_t *__restrict__ skip) {
    using T = typename Ar::T;
    static_assert(sizeof(T) == 4, "4-byte elements");
    constexpr int TT = flow_tile<BS>();
    using PS = P1S<Ar, BS, TT>;
    static_assert(PS::NTH == kSingleThreads && PS::TM1 == TT && PS::TN1 == TT, "TT x TT per thread");
    if (skip && *skip != APSP_SUCCESS) return;
    __shared__ alignas(16) T la[BS * BS];
    __shared__ alignas(16) T lb[BS * BS];
    __shared__ alignas(16) T p1c[4][BS];
    __shared__ alignas(16) T p1r[4][BS];
    __shared__ int ok_lds;
    __shared__ uint32_t ticket_lds;
    T *const X = (T *)Xv;
    T *const Prow = (T *)prow_v;
    T *const Pcol = (T *)pcol_v;
    const uint32_t ordu = (uint32_t)order, stru = (uint32_t)stride;
    const int R = (int)(order / BS);
    const int tid = (int)threadIdx.x, tx = tid % PS::TX, ty = tid / PS::TX;
    uint32_t *const ver = words;
    uint32_t *const fail = words + task_fail_word(R);
    const uint32_t total = (uint32_t)task_count(R);
    auto blk = [&](T *M, uint32_t ld, int p, int q) __attribute__((always_inline)) {
        return M + ((uint32_t)p * BS * ld + (uint32_t)q * BS);
    };
    auto at = [&](T *M, uint32_t ld, int p, int q) __attribute__((always_inline)) {
        return blk(M, ld, p, q) + ((uint32_t)ty * TT * ld + (uint32_t)tx * TT);
    };
    T c[TT][TT];
    bool big = false;
    auto load = [&](int i, int j) __attribute__((always_inline)) {
        T *const src = at(X, stru, i, j);
#pragma unroll
        for (int q = 0; q < TT; ++q) ld_tt_dev<TT>(src + (uint32_t)q * stru, c[q]);
        big |= any_big(ar, c);
    };
    auto multiply = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // this wavefront's copies: vmcnt(0)
        __syncthreads();
#pragma unroll 2
        for (int kg = 0; kg < BS; kg += 4) {
            T a[TT][4];
#pragma unroll
            for (int q = 0; q < TT; ++q) {
                const int row = ty * TT + q;
                ld16(&la[row * BS + (((kg >> 2) ^ flow_swz<BS>(row)) << 2)], a[q]);
            }
#pragma unroll
            for (int kk = 0; kk < 4; kk += 2) {
                T b0[TT], b1[TT];
                ld_tt<TT>(&lb[(kg + kk) * BS + tx * TT], b0);
                ld_tt<TT>(&lb[(kg + kk + 1) * BS + tx * TT], b1);
#pragma unroll
                for (int q = 0; q < TT; ++q)
#pragma unroll
                    for (int n = 0; n < TT; ++n) c[q][n] = ar.relax2(c[q][n], a[q][kk], b0[n], a[q][kk + 1], b1[n]);
            }
        }
    };
    // stores the block state (and its publication, if any), then, once every
    // wavefront's stores are complete, advances ver(i, j) to v
    auto finish = [&](int i, int j, T *pub, uint32_t v) __attribute__((always_inline)) {
        big |= any_big(ar, c);
        T *const dst = at(X, stru, i, j);
#pragma unroll
        for (int q = 0; q < TT; ++q) st_tt_dev<TT>(dst + (uint32_t)q * stru, c[q]);
        if (pub) {
            T *const pd = at(pub, ordu, i, j);
#pragma unroll
            for (int q = 0; q < TT; ++q) st_tt_dev<TT>(pd + (uint32_t)q * ordu, c[q]);
        }
        mem_done();
        __syncthreads();
        if (tid == 0) st_agent(&ver[i * R + j], v);
    };
    auto close = [&]() __attribute__((always_inline)) {
        big |= phase1_steps<Ar, BS, false, TT>(c, BS, ar, p1c, p1r);
    };

    bool ok = true;
    for (;;) {
        __syncthreads();  // LDS (operands, ticket) free for the next task
        if (tid == 0)
            ticket_lds = __hip_atomic_fetch_add(&words[task_next_word(R)], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t t = ticket_lds;
        if (t >= total) break;
        if (!ok) continue;  // after a failed wait: drain the counter, do nothing
        const FlowTask k = task_decode(t, R);
        const int r = k.r, i = k.i, j = k.j;
        if (k.kind == 0) {
            load(0, 0);
            close();
            finish(0, 0, Prow, 1u);
            continue;
        }
        // its own round r - 1 (loaded while the operands are awaited)
        if (!(ok = task_wait(&ver[i * R + j], (uint32_t)r, nullptr, 0u, fail, &ok_lds))) continue;
        load(i, j);
        if (k.kind != 3) {
            // a panel: the closed block r
            if (!(ok = task_wait(&ver[r * R + r], (uint32_t)r + 1, nullptr, 0u, fail, &ok_lds))) continue;
            if (k.kind == 1) {  // c <- min(c, D(r,r)* (x) c)
                flow_copy<BS, kSingleThreads, true>(la, blk(Prow, ordu, r, r), ordu);
#pragma unroll
                for (int q2 = 0; q2 < TT; ++q2) st_tt<TT>(&lb[(ty * TT + q2) * BS + tx * TT], c[q2]);
            } else {  // c <- min(c, c (x) D(r,r)*)
                flow_copy<BS, kSingleThreads, false>(lb, blk(Prow, ordu, r, r), ordu);
#pragma unroll
                for (int q2 = 0; q2 < TT; ++q2) {
                    const int rw = ty * TT + q2, col = tx * TT;
                    st_tt<TT>(&la[rw * BS + (((col >> 2) ^ flow_swz<BS>(rw)) << 2) + (col & 3)], c[q2]);
                }
            }
            multiply();
            finish(i, j, k.kind == 1 ? Prow : Pcol, (uint32_t)r + 1);
            continue;
        }
        // a remaining block: c <- min(c, P_col(i, r) (x) P_row(r, j))
        if (!(ok = task_wait(&ver[i * R + r], (uint32_t)r + 1, &ver[r * R + j], (uint32_t)r + 1, fail, &ok_lds)))
            continue;
        flow_copy<BS, kSingleThreads, true>(la, blk(Pcol, ordu, i, r), ordu);
        flow_copy<BS, kSingleThreads, false>(lb, blk(Prow, ordu, r, j), ordu);
        multiply();
        if (i == r + 1 && j == r + 1) {
            close();
            finish(i, j, Prow, (uint32_t)r + 2);
        } else {
            finish(i, j, nullptr, (uint32_t)r + 1);
        }
    }
    if constexpr (Ar::kWatch) {
        if (big && tid == 0) ar.raise();
    }
    if (!ok && status && tid == 0) *status = APSP_ERROR_TIMEOUT;
    // the last workgroup to finish clears the words for the next launch
    __syncthreads();
    if (tid == 0)
        ok_lds = __hip_atomic_fetch_add(&words[task_done_word(R)], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
                 gridDim.x - 1;
    __syncthreads();
    if (ok_lds)
        for (int k = tid; k < task_words(R); k += kSingleThreads) st_agent(&words[k], 0u);
}

// ------------------------------------------------------ set-up / wrap-up
__global__ void status_init_kernel(int32_t *status) { *status = APSP_SUCCESS; }

// Checks the weight preconditions of the public header.
template <class T>
__global__ void validate_kernel(const T *__restrict__ W, int64_t n, int64_t bound,
                                int32_t *__restrict__ status) {
    const int64_t total = n * n;
    bool bad = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        const T w = W[e];
        if constexpr (std::is_same_v<T, float>) {
            if (w != w || w == -__builtin_inff()) bad = true;
            if (i == j && w != 0.0f) bad = true;
        } else {
            if (i == j) {
                if (w != 0) bad = true;
            } else if (w != kInf32 && (w > bound || w < -bound)) {
                bad = true;
            }
        }
    }
    if (bad) *status = APSP_ERROR_INVALID_VALUE;
}

// Copies the caller's n x n matrix into the ld x ld work matrix; padding
// vertices are isolated (INF off the diagonal, 0 on it).
template <class T>
__global__ void pad_in_kernel(const T *__restrict__ W, int64_t n, T *__restrict__ X, int64_t ld,
                              T inf, const int32_t *__restrict__ skip) {
    if (skip && *skip != APSP_SUCCESS) return;
    const int64_t total = ld * ld;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ld, j = e - i * ld;
        T v;
        if (i < n && j < n)
            v = W[i * n + j];
        else
            v = (i == j) ? T(0) : inf;
        X[e] = v;
    }
}

// Distance-only wrap-up: map int32 sums that carried the sentinel back to
// INF, copy to the caller's buffer when a padded work matrix was used, and
// report a negative cycle (a negative diagonal, or an int32 value below
// kWrapWitness).
template <class T>
__global__ void finalize_kernel(const T *__restrict__ X, int64_t ld, T *__restrict__ out, int64_t n,
                                int32_t *__restrict__ status, const int32_t *__restrict__ skip) {
    if (skip && *skip != APSP_SUCCESS) return;
    const int64_t total = n * n;
    bool neg = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        T v = X[i * ld + j];
        if constexpr (std::is_same_v<T, int32_t>) {
            if (v < kWrapWitness) neg = true;
            if (v >= kFakeThreshold) v = kInf32;
        }
        if (i == j && v < T(0)) neg = true;
        out[e] = v;
    }
    if (neg && status) *status = APSP_ERROR_NEGATIVE_CYCLE;
}

// The same for float32 distances solved in the caller's buffer: nothing to
// map or copy, so only the diagonal is read.
__global__ void finalize_diag_kernel(const float *__restrict__ X, int64_t ld, int64_t n, int32_t *__restrict__ status,
                                     const int32_t *__restrict__ skip) {
    if (skip && *skip != APSP_SUCCESS) return;
    bool neg = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (X[i * ld + i] < 0.0f) neg = true;
    if (neg && status) *status = APSP_ERROR_NEGATIVE_CYCLE;
}

// int32 distance solves in float32 arithmetic (policy ArF32W).  words[0]:
// set when a watched value reached 2^23 (the float32 result may then be
// inexact and is discarded); words[1]: gate of the int32 pass that follows
// (APSP_SUCCESS = run it, anything else = skip).
__global__ void f32w_init_kernel(int32_t *words) {
    words[0] = 0;
    words[1] = 1;
}

// Converts the caller's int32 weights into the ld x ld float32 work matrix
// (INF -> +inf, padding vertices isolated); weights of magnitude >= 2^23 set
// words[0] right away.
// Row-wise element loops: blockIdx.y strides rows, each thread four
// consecutive columns (ld is a multiple of the block size, so of 4).
__device__ __forceinline__ float f32w_in_one(int32_t w, bool &big) {
    if (w == kInf32) return __builtin_inff();
    big |= (w >= (1 << 23) || w <= -(1 << 23));
    return (float)w;
}

// vec: the caller's rows start on 16-byte boundaries (n % 4 == 0, aligned W)
__global__ void f32w_in_kernel(const int32_t *__restrict__ W, int64_t n, float *__restrict__ X, int64_t ld,
                               int32_t *__restrict__ words, const int32_t *__restrict__ skip, int vec) {
    if (skip && *skip != APSP_SUCCESS) return;
    bool big = false;
    for (int64_t i = blockIdx.y; i < ld; i += gridDim.y) {
        for (int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; j < ld;
             j += (int64_t)gridDim.x * blockDim.x * 4) {
            float v[4];
            if (vec && i < n && j + 4 <= n) {
                const int4 w = *reinterpret_cast<const int4 *>(W + i * n + j);
                v[0] = f32w_in_one(w.x, big);
                v[1] = f32w_in_one(w.y, big);
                v[2] = f32w_in_one(w.z, big);
                v[3] = f32w_in_one(w.w, big);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t jj = j + q;
                    if (i < n && jj < n)
                        v[q] = f32w_in_one(W[i * n + jj], big);
                    else
                        v[q] = (i == jj) ? 0.0f : __builtin_inff();  // padding vertices are isolated
                }
            }
            *reinterpret_cast<float4 *>(X + i * ld + j) = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
    if (big) words[0] = 1;
}

// If no watcher fired, the float32 result is the exact int32 result:
// write it back (+inf -> INF) and report a negative diagonal.
__global__ void f32w_out_kernel(const float *__restrict__ X, int64_t ld, int32_t *__restrict__ out, int64_t n,
                                int32_t *__restrict__ status, const int32_t *__restrict__ words,
                                const int32_t *__restrict__ skip, int vec) {
    if (skip && *skip != APSP_SUCCESS) return;
    if (words[0]) return;
    bool neg = false;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        for (int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; j < n;
             j += (int64_t)gridDim.x * blockDim.x * 4) {
            const float4 x = *reinterpret_cast<const float4 *>(X + i * ld + j);  // j + 3 < ld
            const float v[4] = {x.x, x.y, x.z, x.w};
            int32_t o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o[q] = (v[q] == __builtin_inff()) ? kInf32 : (int32_t)v[q];
                if (i == j + q && v[q] < 0.0f) neg = true;
            }
            if (vec && j + 4 <= n) {
                *reinterpret_cast<int4 *>(out + i * n + j) = make_int4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (j + q < n) out[i * n + j + q] = o[q];
            }
        }
    }
    if (neg && status) *status = APSP_ERROR_NEGATIVE_CYCLE;
}

// Opens the int32 pass when the float32 pass was not exact; reports the
// arithmetic that produced the result (1 = float32, 0 = int32).
__global__ void f32w_gate_kernel(int32_t *words, const int32_t *__restrict__ skip, int32_t *arith_used) {
    const bool ok = !(skip && *skip != APSP_SUCCESS);
    const bool redo = ok && words[0] != 0;
    words[1] = redo ? APSP_SUCCESS : 1;
    if (arith_used) *arith_used = (ok && !redo) ? 1 : 0;
}

__global__ void store_word_kernel(int32_t *p, int32_t v) {
    if (p) *p = v;
}

// Predecessor solves.  mode == nullptr or *mode == 0: key mode,
// key = d * 2^S + p (p = i for an edge i->j, i != j, else 2^S - 1 = none;
// +inf when absent).  *mode != 0 (float32 weights that are not all
// integers within the bound): (distance, predecessor) pairs.
__global__ void mode_init_kernel(int32_t *mode) { *mode = 0; }

// Sets *mode = 1 if some finite off-diagonal float32 weight is not an
// integer of magnitude <= bound (key arithmetic would then not be exact).
__global__ void integral_check_kernel(const float *__restrict__ W, int64_t n, float bound,
                                      int32_t *__restrict__ mode) {
    const int64_t total = n * n;
    bool lex = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float w = W[e];
        if (w == __builtin_inff()) continue;
        if (w != __builtin_floorf(w) || __builtin_fabsf(w) > bound) lex = true;
    }
    if (lex) *mode = 1;
}

template <class T>
__global__ void pred_pack_kernel(const T *__restrict__ W, int64_t n, void *__restrict__ Xv,
                                 int64_t ld, int S, const int32_t *__restrict__ mode,
                                 const int32_t *__restrict__ skip) {
    if (skip && *skip != APSP_SUCCESS) return;
    const bool lex = mode && *mode;
    const int64_t total = ld * ld;
    const double none = (double)((1 << S) - 1);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ld, j = e - i * ld;
        bool absent = i != j;
        double w = 0.0;
        if (i < n && j < n) {
            const T x = W[i * n + j];
            if constexpr (std::is_same_v<T, int32_t>)
                absent = (x == kInf32);
            else
                absent = (x == __builtin_inff());
            w = (double)x;
        }
        const bool edge = !absent && i != j;
        if (lex) {
            DistPred v{absent ? __builtin_inff() : (float)w, edge ? (int32_t)i : kLexNone};
            ((DistPred *)Xv)[e] = v;
        } else {
            ((double *)Xv)[e] = absent ? __builtin_inf() : __builtin_ldexp(w, S) + (edge ? (double)i : none);
        }
    }
}

template <class T>
__global__ void pred_unpack_kernel(const void *__restrict__ Xv, int64_t ld, T *__restrict__ dist,
                                   int32_t *__restrict__ pred, int64_t n, int S,
                                   const int32_t *__restrict__ mode, int32_t *__restrict__ status,
                                   const int32_t *__restrict__ skip) {
    if (skip && *skip != APSP_SUCCESS) return;
    const bool lex = mode && *mode;
    const int64_t total = n * n;
    const int32_t none = (1 << S) - 1;
    bool neg = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        T d;
        int32_t p;
        bool unreachable;
        if (lex) {
            const DistPred v = ((const DistPred *)Xv)[i * ld + j];
            unreachable = v.d == __builtin_inff();
            d = (T)v.d;
            p = (v.p == kLexNone) ? APSP_NO_PRED : v.p;
            if (i == j && v.d < 0.0f) neg = true;
        } else {
            const double key = ((const double *)Xv)[i * ld + j];
            unreachable = key == __builtin_inf();
            const double dd = unreachable ? 0.0 : __builtin_floor(__builtin_ldexp(key, -S));
            p = unreachable ? APSP_NO_PRED : (int32_t)(key - __builtin_ldexp(dd, S));
            d = (T)dd;
            if (p == none) p = APSP_NO_PRED;
            if (i == j && dd < 0.0) neg = true;
        }
        if (unreachable) {
            if constexpr (std::is_same_v<T, int32_t>)
                d = kInf32;
            else
                d = __builtin_inff();
            p = APSP_NO_PRED;
        }
        if (i == j) p = APSP_NO_PRED;
        dist[e] = d;
        if (pred) pred[e] = p;
    }
    if (neg && status) *status = APSP_ERROR_NEGATIVE_CYCLE;
}

// ------------------------------------ predecessors from final distances
// With exact distances D, the canonical predecessor has the closed form
//     P(i,j) = min{v != j : W(v,j) finite, D(i,v) + W(v,j) = D(i,j)}
// (the fixed point of the lexicographic recurrence), and
//     D(i,j) * 2^S + P(i,j) = min_v [(D(i,v) * 2^S + v) + W(v,j) * 2^S]
// over v != j (S bits hold any vertex).  So a solve that needs predecessors
// can compute the distances in exact float32 arithmetic (ArF32W) and then
// read P off one float32 min-plus product of A(i,v) = D(i,v) 2^S + v with
// B(v,j) = W(v,j) 2^S (B(j,j) = +inf), in place of the fp64-key recurrence.
// The product is exact when A and B are: every B entry is (|W| < 2^23),
// and an A entry of magnitude >= 2^24 can only lose when all weights are
// non-negative (its candidates then stay >= 2^24 above every in-range
// key).  The winning key must lie below 2^24 in magnitude and its distance
// part must equal D(i,j).  Anything else raises a word and the device runs
// the fp64-key recurrence on the original weights instead.
//
// words (int32): see kPP* below.  APSP_SUCCESS in kPPGate opens the
// fallback; APSP_SUCCESS in kPPRounds opens the float32 distance rounds.
constexpr int kPPBig = 0;       // a watched float32 value reached 2^23 (ArF32W)
constexpr int kPPGate = 1;      // fallback gate
constexpr int kPPMode = 2;      // float32 weights not all integers within the bound: pairs
constexpr int kPPReject = 3;    // a non-zero diagonal entry
constexpr int kPPNegW = 4;      // some finite off-diagonal weight is negative
constexpr int kPPPosBig = 5;    // some finite A entry >= 2^24
constexpr int kPPNegBig = 6;    // some finite A entry <= -2^24
constexpr int kPPFail = 7;      // the product's check failed for some (i,j)
constexpr int kPPWritten = 8;   // dist holds distances (the weights must be restored)
constexpr int kPPSkip = 9;      // the product does not run
constexpr int kPPRounds = 10;   // gate of the float32 distance rounds
constexpr int kPPWords = 11;

__global__ void pp_init_kernel(int32_t *words) {
    for (int q = 0; q < kPPWords; ++q) words[q] = 0;
    words[kPPGate] = 1;
    words[kPPRounds] = 1;
}

template <class T>
__device__ __forceinline__ void pp_in_one(T w, bool diag, float bound, float scale, float &x, float &b,
                                          bool &big, bool &mode, bool &reject, bool &negw) {
    bool fin;
    float wf;
    if constexpr (std::is_same_v<T, int32_t>) {
        fin = w != kInf32;
        wf = (float)w;
        if (fin && (w >= (1 << 23) || w <= -(1 << 23))) big = true;
    } else {
        fin = w != __builtin_inff();
        wf = w;
        if (fin && (w != __builtin_floorf(w) || __builtin_fabsf(w) > bound)) mode = true;  // NaN too
        if (fin && __builtin_fabsf(w) >= 8388608.0f) big = true;
    }
    if (diag) {
        if (!(w == T(0))) reject = true;
        x = 0.0f;
        b = __builtin_inff();
    } else {
        x = fin ? wf : __builtin_inff();
        b = fin ? wf * scale : __builtin_inff();
        if (fin && wf < 0.0f) negw = true;
    }
}

// W (n x n, caller's) -> X (float32 distances to be, ld x ld, padding
// vertices isolated) and B = W 2^S with +inf on the diagonal and padding.
template <class T>
__global__ void pp_in_kernel(const T *__restrict__ W, int64_t n, float *__restrict__ X, float *__restrict__ Bm,
                             int64_t ld, int S, float bound, int32_t *__restrict__ words,
                             const int32_t *__restrict__ skip, int vec) {
    if (skip && *skip != APSP_SUCCESS) return;
    const float scale = __builtin_ldexpf(1.0f, S);
    bool big = false, mode = false, reject = false, negw = false;
    for (int64_t i = blockIdx.y; i < ld; i += gridDim.y) {
        for (int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; j < ld;
             j += (int64_t)gridDim.x * blockDim.x * 4) {
            float x[4], b[4];
            if (vec && i < n && j + 4 <= n) {
                T w[4];
                if constexpr (std::is_same_v<T, int32_t>) {
                    const int4 v = *reinterpret_cast<const int4 *>(W + i * n + j);
                    w[0] = v.x, w[1] = v.y, w[2] = v.z, w[3] = v.w;
                } else {
                    const float4 v = *reinterpret_cast<const float4 *>(W + i * n + j);
                    w[0] = v.x, w[1] = v.y, w[2] = v.z, w[3] = v.w;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    pp_in_one<T>(w[q], i == j + q, bound, scale, x[q], b[q], big, mode, reject, negw);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t jj = j + q;
                    if (i < n && jj < n) {
                        pp_in_one<T>(W[i * n + jj], i == jj, bound, scale, x[q], b[q], big, mode, reject, negw);
                    } else {
                        x[q] = (i == jj) ? 0.0f : __builtin_inff();
                        b[q] = __builtin_inff();
                    }
                }
            }
            *reinterpret_cast<float4 *>(X + i * ld + j) = make_float4(x[0], x[1], x[2], x[3]);
            *reinterpret_cast<float4 *>(Bm + i * ld + j) = make_float4(b[0], b[1], b[2], b[3]);
        }
    }
    if (big) words[kPPBig] = 1;
    if (mode) words[kPPMode] = 1;
    if (reject) words[kPPReject] = 1;
    if (negw) words[kPPNegW] = 1;
}

// Opens the float32 distance rounds unless the weights already rule the
// product out (pairs needed, or a non-zero diagonal).
__global__ void pp_rounds_gate_kernel(int32_t *words, const int32_t *__restrict__ skip) {
    const bool ok = !(skip && *skip != APSP_SUCCESS);
    words[kPPRounds] = (ok && !words[kPPMode] && !words[kPPReject]) ? APSP_SUCCESS : 1;
}

// If the float32 distances are exact: writes them to dist (+inf -> INF for
// int32), reports a negative diagonal, and turns X into A in place:
// A(i,v) = X(i,v) 2^S + v (+inf stays +inf; padding columns are +inf).
template <class T>
__global__ void pp_out_kernel(float *__restrict__ X, int64_t ld, T *__restrict__ dist, int64_t n, int S,
                              int32_t *__restrict__ words, int32_t *__restrict__ status,
                              const int32_t *__restrict__ skip, int vec) {
    if (skip && *skip != APSP_SUCCESS) return;
    if (words[kPPBig] || words[kPPRounds] != APSP_SUCCESS) return;
    bool neg = false, posbig = false, negbig = false;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        for (int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; j < n;
             j += (int64_t)gridDim.x * blockDim.x * 4) {
            float4 *px = reinterpret_cast<float4 *>(X + i * ld + j);  // j + 3 < ld
            const float4 xv = *px;
            const float x[4] = {xv.x, xv.y, xv.z, xv.w};
            T o[4];
            float a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool fin = x[q] != __builtin_inff();
                if constexpr (std::is_same_v<T, int32_t>)
                    o[q] = fin ? (int32_t)x[q] : kInf32;
                else
                    o[q] = x[q];
                if (i == j + q && x[q] < 0.0f) neg = true;
                if (fin) {
                    const double kd = __builtin_ldexp((double)x[q], S) + (double)(j + q);
                    posbig |= kd >= 16777216.0;
                    negbig |= kd <= -16777216.0;
                    a[q] = (float)kd;
                } else {
                    a[q] = __builtin_inff();
                }
            }
            *px = make_float4(a[0], a[1], a[2], a[3]);
            if (vec && j + 4 <= n) {
                if constexpr (std::is_same_v<T, int32_t>)
                    *reinterpret_cast<int4 *>(dist + i * n + j) = make_int4(o[0], o[1], o[2], o[3]);
                else
                    *reinterpret_cast<float4 *>(dist + i * n + j) = make_float4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (j + q < n) dist[i * n + j + q] = o[q];
            }
        }
    }
    if (threadIdx.x == 0) words[kPPWritten] = 1;
    if (posbig) words[kPPPosBig] = 1;
    if (negbig) words[kPPNegBig] = 1;
    if (neg && status) *status = APSP_ERROR_NEGATIVE_CYCLE;
}

// Decides whether the product runs (its keys would be exact).
__global__ void pp_product_gate_kernel(int32_t *words) {
    const bool no = words[kPPBig] || words[kPPRounds] != APSP_SUCCESS || words[kPPNegBig] ||
                    (words[kPPPosBig] && words[kPPNegW]);
    words[kPPSkip] = no ? 1 : 0;
}

// P(i,j) from min_v A(i,v) + B(v,j) over v < kcount, 128 x 128 output tiles
// (the 8 x 8 register blocks and LDS DMA staging of phase 3), tiles grouped
// 8 rows at a time and split over the XCDs in contiguous stretches.
template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kP3Waves4)))
pp_product_kernel(const float *__restrict__ A, const float *__restrict__ Bm, int64_t ld, int kcount,
                  const T *__restrict__ dist, int32_t *__restrict__ pred, int64_t n, int S, int nt, int per_xcd,
                  int32_t *__restrict__ words, const int32_t *__restrict__ skip) {
    using TP = TileProductDMA<ArF32, 128, 128, 16, 8, 8>;
    static_assert(TP::NTH == 256 && TP::TX == 16 && TP::TY == 16 && TP::GN == 2, "tile shape");
    if (skip && *skip != APSP_SUCCESS) return;
    if (words[kPPSkip]) return;
    constexpr int GROUP = 8;
    const int w = blockIdx.x;
    const int seq = (w & 7) * per_xcd + (w >> 3);
    if (seq >= nt * nt) return;
    const int group = seq / (GROUP * nt);
    const int first = group * GROUP;
    const int rows = min(GROUP, nt - first);
    const int within = seq - group * GROUP * nt;
    const int64_t crow = (int64_t)(first + within % rows) * 128;
    const int64_t ccol = (int64_t)(within / rows) * 128;
    __shared__ typename TP::Smem sm;
    const int tx = threadIdx.x % TP::TX, ty = threadIdx.x / TP::TX;
    float c[8][8];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < 8; ++q) c[m][q] = __builtin_inff();
    TP::accumulate(sm, c, A + crow * ld, Bm + ccol, (uint32_t)ld, kcount, tx, ty, ArF32{});
    const float down = __builtin_ldexpf(1.0f, -S), up = __builtin_ldexpf(1.0f, S);
    bool fail = false;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int64_t i = crow + ty + TP::TY * m;
        if (i >= n) continue;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t j = ccol + (q / 4) * TP::GSTRIDE + tx * 4 + (q % 4);
            if (j >= n) continue;
            const T d = dist[i * n + j];
            bool reach;
            if constexpr (std::is_same_v<T, int32_t>)
                reach = d != kInf32;
            else
                reach = d != __builtin_inff();
            int32_t p = APSP_NO_PRED;
            if (i != j && reach) {
                const float key = c[m][q];
                if (__builtin_fabsf(key) < 16777216.0f) {
                    const float kd = __builtin_floorf(key * down);
                    if (kd == (float)d)
                        p = (int32_t)(key - kd * up);
                    else
                        fail = true;
                } else {
                    fail = true;  // also +inf: no candidate although D(i,j) is finite
                }
            }
            pred[i * n + j] = p;
        }
    }
    if (fail) words[kPPFail] = 1;
}

// Opens the fp64-key fallback when the product did not run or failed its
// check; reports the arithmetic that produced the result (1 = float32
// distances + product, 0 = the exact key recurrence).
__global__ void pp_gate_kernel(int32_t *words, const int32_t *__restrict__ skip, int32_t *arith_used) {
    const bool ok = !(skip && *skip != APSP_SUCCESS);
    const bool redo = ok && (words[kPPSkip] || words[kPPFail]);
    words[kPPGate] = redo ? APSP_SUCCESS : 1;
    if (arith_used) *arith_used = (ok && !redo) ? 1 : 0;
}

// Fallback after dist was overwritten: the weights back from B (exact: every
// weight was an integer below 2^23), zero diagonal.
template <class T>
__global__ void pp_restore_kernel(const float *__restrict__ Bm, int64_t ld, T *__restrict__ dist, int64_t n, int S,
                                  const int32_t *__restrict__ words) {
    if (words[kPPGate] != APSP_SUCCESS || !words[kPPWritten]) return;
    const float down = __builtin_ldexpf(1.0f, -S);
    const int64_t total = n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        const float b = Bm[i * ld + j];
        T w;
        if (i == j)
            w = T(0);
        else if (b == __builtin_inff())
            w = std::is_same_v<T, int32_t> ? T(kInf32) : T(__builtin_inff());
        else
            w = (T)(b * down);
        dist[e] = w;
    }
}

// --------------------------------------------------------------- runtime
namespace {

thread_local int g_last_hip = 0;

struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

#define APSP_HIP(call)                                    \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) {                           \
            g_last_hip = (int)e_;                         \
            return APSP_ERROR_HIP;                        \
        }                                                 \
    } while (0)

// Device workspace private to (device, stream): work on one stream is
// ordered, so reusing it across calls on that stream is race-free.
apsp_status_t cached_workspace(int dev, hipStream_t s, size_t bytes, void **out) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, s}];
    if (w.bytes < bytes) {
        if (w.ptr) {
            APSP_HIP(hipStreamSynchronize(s));
            APSP_HIP(hipFree(w.ptr));
            w.ptr = nullptr;
            w.bytes = 0;
        }
        hipError_t e = hipMalloc(&w.ptr, bytes);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            w.ptr = nullptr;
            return APSP_ERROR_OUT_OF_MEMORY;
        }
        w.bytes = bytes;
    }
    *out = w.ptr;
    return APSP_SUCCESS;
}

// Optional per-launch timing (apsp_profile_begin / _end).
enum KernelKind {
    kPhase1 = 0,
    kPhase2 = 1,
    kPhase3 = 2,
    kOther = 3,
    kPhase3Cross = 4,
    kPredProduct = 5,
    kPhase1Blocked = 6,  // counted under phase1 and phase1_blocked
    kSingle = 7,         // the single-launch schedule's one kernel
    kPhase1Flow = 8      // counted under phase1 and phase1_flow
};
struct ProfRecord {
    int kind;
    double updates;
    hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;

thread_local bool t_capturing = false;  // launches are being recorded into a hipGraph
thread_local bool t_noalloc = false;    // apsp_solve_noalloc: no event creation either

// Operations of a solve recorded for a stepper (see enq below).
struct Recorder {
    std::vector<std::function<hipError_t()>> ops;
    std::vector<size_t> marks;  // index of the first operation of each round
};
struct AuxStream;
thread_local Recorder *t_rec = nullptr;
thread_local AuxStream *t_aux = nullptr;  // the recording stepper's second stream

struct ProfScope {
    ProfRecord rec{};
    hipStream_t s;
    bool on;
    ProfScope(int kind, double updates, hipStream_t stream) : s(stream) {
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            on = g_prof_on && !t_capturing && !t_rec && !t_noalloc && kind >= 0;
        }
        if (!on) return;
        rec.kind = kind;
        rec.updates = updates;
        if (hipEventCreate(&rec.start) != hipSuccess || hipEventCreate(&rec.stop) != hipSuccess) {
            on = false;
            return;
        }
        (void)hipEventRecord(rec.start, s);
    }
    ~ProfScope() {
        if (!on) return;
        (void)hipEventRecord(rec.stop, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back(rec);
    }
};

// Grid of the row-wise element kernels over a rows x cols region (4
// columns per thread, 256 threads per block).
inline dim3 grid_rows(int64_t rows, int64_t cols) {
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>((cols / 4 + 255) / 256, 64));
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(rows, 8192 / gx));
    return dim3((unsigned)gx, (unsigned)gy);
}

inline int grid_for(int64_t elems, int per_block = 256) {
    int64_t g = (elems + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

int pred_bits(int64_t ld) {
    int S = 1;
    while ((int64_t(1) << S) < ld + 1) ++S;
    return S;
}

// Auxiliary stream per (device, caller stream) for the two-stream schedule,
// with the two events it uses.
struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t panels = nullptr;  // caller stream: phase 2 of the current round done
    hipEvent_t rest = nullptr;    // aux stream: kRest tiles of the previous round done
};
std::mutex g_aux_mu;
std::map<std::pair<int, hipStream_t>, AuxStream> g_aux;

void aux_destroy(AuxStream &a) {
    if (a.panels) (void)hipEventDestroy(a.panels);
    if (a.rest) (void)hipEventDestroy(a.rest);
    if (a.s) (void)hipStreamDestroy(a.s);
    a = AuxStream{};
}

apsp_status_t aux_stream(int dev, hipStream_t s, AuxStream **out) {
    std::lock_guard<std::mutex> lk(g_aux_mu);
    AuxStream &a = g_aux[{dev, s}];
    if (!a.s) {
        AuxStream n;  // all three or none
        hipError_t e = hipStreamCreateWithFlags(&n.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.panels, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.rest, hipEventDisableTiming);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            aux_destroy(n);
            return APSP_ERROR_HIP;
        }
        a = n;
    }
    *out = &a;
    return APSP_SUCCESS;
}

// ------------------------------------------------------------ recording
// The launch sequence of a solve never depends on the data (every
// data-dependent choice is a device word), so it can be recorded once and
// issued later in slices: a stepper (apsp_stepper_*) records it, with its
// own work memory and second stream, and issues it a few rounds at a time.
// Without a recorder every operation is issued at once.
template <class K, class... A>
inline void enq(K kernel, dim3 grid, dim3 block, hipStream_t s, A... args) {
    if (t_rec) {
        t_rec->ops.push_back([=]() -> hipError_t {
            hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
            return hipGetLastError();
        });
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}
inline hipError_t enq_record(hipEvent_t e, hipStream_t s) {
    if (!t_rec) return hipEventRecord(e, s);
    t_rec->ops.push_back([=]() { return hipEventRecord(e, s); });
    return hipSuccess;
}
inline hipError_t enq_wait(hipStream_t s, hipEvent_t e) {
    if (!t_rec) return hipStreamWaitEvent(s, e, 0);
    t_rec->ops.push_back([=]() { return hipStreamWaitEvent(s, e, 0); });
    return hipSuccess;
}
inline void round_mark() {
    if (t_rec) t_rec->marks.push_back(t_rec->ops.size());
}

// The round loop on a work matrix of size ld (a multiple of BS).
//
// One stream, in order: for each round r, phase 1, phase 2, phase 3.
// Two streams (lookahead, from three rounds on): phase 3 of round r is
// split into the tiles the next round's phases 1-2 read (kCross, on the
// caller's stream, the critical path) and all others (kRest, on an
// auxiliary stream), so phases 1 and 2 of round r+1 run beside the bulk of
// phase 3 of round r:
//   caller: P1(0) P2(0) [panels] | wait(rest) P3x(r) P1(r+1) P2(r+1) [panels] | ...
//   aux:    wait(panels) P3r(r) [rest] | ...
// kCross(r+1) touches tiles last written by kRest(r), hence its wait.
// A phase-1 workgroup needs most of a compute unit's registers, so it only
// starts where kRest's workgroups drain; kRest is therefore issued as
// kRestChunks launches, whose boundaries let the caller stream's kernels
// in (2 measured best: about 1.4 % at n = 32768, 6 % at n = 16384).
// Schedule choices of one pass of rounds (apsp_options_t.schedule / .phase1:
// 0 automatic by size, 1 rounds in order / the stepwise phase-1 kernel,
// 2 the two-stream split / the blocked phase 1 wherever they apply).
struct Sched {
    int schedule = 0;
    int phase1 = 0;
};

// Phase 1 of 128- and 256-wide blocks as a dataflow closure: the diagonal
// block is solved by the blocked schedule itself, over 32-wide sub-blocks,
// in one launch of (BS/32)^2 workgroups (flow_tasks_kernel on the block in
// place: its order is BS, its row stride ld).  In exact arithmetic (int32,
// and float32 watched for exactness) its values are those of BS single
// steps (real-valued float32: those of the blocked schedule, rounded
// otherwise than the stepwise kernel, within float32 rounding; every way of
// issuing a solve -- direct, hipGraph, stepper, apsp_solve_noalloc -- makes
// the same choice, so they agree bit for bit).  An ordinary launch: its tasks are taken in dependency order, so
// it completes however many of its workgroups are resident beside other
// work (several solves on several streams included).  Per (device, stream)
// scratch: the two 256 x 256 published matrices and the task words, zeroed
// once at allocation (each launch leaves its words zeroed again).
template <class Ar, int BS, class Alt>
constexpr bool kFlowP1 = (BS == 128 || BS == 256) && std::is_same_v<Alt, NoAlt> &&
                         (std::is_same_v<Ar, ArI32> || std::is_same_v<Ar, ArF32W> || std::is_same_v<Ar, ArF32>);
constexpr int kClosureBS = 32, kClosureMax = 256;
constexpr size_t kClosurePub = (size_t)kClosureMax * kClosureMax * 4;
constexpr size_t kClosureBytes = 2 * kClosurePub + task_word_bytes(kClosureMax / kClosureBS);
std::mutex g_closure_mu;
std::map<std::pair<int, hipStream_t>, void *> g_closure;

// The calling stream's closure scratch; allocates it unless `create` is
// false (then *out is null where none exists yet).  Its words are zeroed
// by a kernel on that stream, so the zeros precede every launch that uses
// them (a memset on the null stream would not be ordered before work on a
// non-blocking stream).
apsp_status_t closure_scratch(int dev, hipStream_t s, bool create, void **out) {
    std::lock_guard<std::mutex> lk(g_closure_mu);
    void *&p = g_closure[{dev, s}];
    if (!p && create) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, kClosureBytes);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            return APSP_ERROR_OUT_OF_MEMORY;
        }
        const int words = (int)((kClosureBytes - 2 * kClosurePub) / 4);
        hipLaunchKernelGGL(flow_init_kernel, dim3(1), dim3(256), 0, s, (uint32_t *)((char *)q + 2 * kClosurePub),
                           words, (int32_t *)nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            (void)hipFree(q);
            return APSP_ERROR_HIP;
        }
        p = q;
    }
    *out = p;
    return APSP_SUCCESS;
}

thread_local int32_t *t_status = nullptr;  // the solve's status word (timeouts of the closure)
// closure scratch of a stepper's recording (its own work memory; the words
// are zeroed inside the recorded sequence) or of apsp_solve_noalloc (a
// slice of the static array, zero from load and left zeroed by each launch)
thread_local void *t_closure = nullptr;

template <class Ar, class Alt, int BS, int TT>
apsp_status_t run_rounds(void *X, int64_t ld, const Ar &ar, const Alt &alt, const int32_t *mode,
                         hipStream_t s, const int32_t *skip, Sched sc, bool prof) {
    constexpr int MT = BS >= 128 ? 128 : 64;
    constexpr int P2W = 64;
    const int R = (int)(ld / BS);
    const int nt2 = (int)((ld - BS) / P2W);
    const int nt = (int)(ld / MT), pb = BS / MT;
    const double bs3 = (double)BS * BS * BS;
    int dev = 0;
    APSP_HIP(hipGetDevice(&dev));
    AuxStream *aux = nullptr;
    // the split pays off once phase 3 is throughput- rather than latency-bound:
    // from ld = 4096 for 4-byte elements, from 3072 for fp64 keys (measured
    // on MI355X with predecessors: 3.58 vs 3.88 ms at n = 3072, 5.12 vs 5.32
    // at 3584, slower at 2048; distances alone lose below 4096)
    // (schedule 2 forces the split at any size with three rounds or more)
    const int64_t split_from = sizeof(typename Ar::T) == 8 ? 3072 : 4096;
    if (sc.schedule != 1 && R >= 3 && (sc.schedule == 2 || ld >= split_from)) {
        if (t_aux) {
            aux = t_aux;
        } else {
            apsp_status_t st = aux_stream(dev, s, &aux);
            if (st != APSP_SUCCESS) return st;
        }
    }
    // the blocked closure is slower on its own (one wavefront per SIMD) but
    // starts in any slot a phase-3 workgroup frees: it pays off where
    // phase 3 is long enough to hide it (measured on MI355X: -4 to -6 % at
    // n = 10240 ... 12288, -3 % at 16384, -0.4 % at 32768; +7 % at 9216 and
    // +23 % at 8192)
    constexpr bool kBlockedP1 = BS == 256 && sizeof(typename Ar::T) == 4 && std::is_same_v<Alt, NoAlt>;
    // The dataflow closure (phase1 3, and the automatic choice for 4-byte
    // distances: measured on MI355X, int32 distances, ms per solve against the
    // stepwise kernel / the blocked closure: n = 6144 8.68 / 9.39; 8192
    // 15.77 / 17.36; 10240 29.16 / 31.36 / 29.67; 16384 111.2 / 113.8 /
    // 112.0; 32768 882.0 / - / 886.1).  Its scratch: a stepper's or
    // apsp_solve_noalloc's own (t_closure), else the stream's (made before
    // any graph capture that may need it).
    void *closure = nullptr;
    if constexpr (kFlowP1<Ar, BS, Alt>) {
        if (sc.phase1 == 3 || sc.phase1 == 0) {
            if (t_closure) {
                closure = t_closure;
                if (t_rec)  // a stepper's recording: zero the words at the start of this pass
                    enq(flow_init_kernel, dim3(1), dim3(256), s, (uint32_t *)((char *)closure + 2 * kClosurePub),
                        (int)((kClosureBytes - 2 * kClosurePub) / 4), (int32_t *)nullptr);
            } else if (!t_noalloc && !t_rec) {
                apsp_status_t st = closure_scratch(dev, s, !t_capturing, &closure);
                if (st != APSP_SUCCESS) return st;
            }
        }
    }
    // (phase1 2 forces it wherever it applies, 1 keeps the stepwise kernel)
    const bool blocked_p1 = kBlockedP1 && (sc.phase1 == 2 || (sc.phase1 == 0 && ld >= 10240 && !closure));
    auto p1 = [&](int r) {
        ProfScope ps(!prof ? -1 : blocked_p1 ? kPhase1Blocked : closure ? kPhase1Flow : kPhase1, bs3, s);
        if constexpr (kFlowP1<Ar, BS, Alt>) {
            if (closure) {
                constexpr int RC = BS / kClosureBS;
                char *const c = (char *)closure;
                enq((flow_tasks_kernel<Ar, kClosureBS>), dim3(RC * RC), dim3(kSingleThreads), s,
                    (void *)((typename Ar::T *)X + (int64_t)r * BS * ld + (int64_t)r * BS), (int64_t)BS, ld, ar,
                    (uint32_t *)(c + 2 * kClosurePub), (void *)c, (void *)(c + kClosurePub), t_status, skip);
                return;
            }
        }
        if (blocked_p1) {
            if constexpr (kBlockedP1)
                enq((phase1_blocked_kernel<Ar>), dim3(1), dim3(256), s, X, ld, (int64_t)r * BS,
                                   ar, skip);
        } else {
            enq((phase1_kernel<Ar, Alt, BS, TT>), dim3(1), dim3(P1S<Ar, BS, TT>::NTH), s, X,
                               ld, (int64_t)r * BS, ar, alt, mode, skip);
        }
    };
    auto p2 = [&](int r) {
        if (nt2 <= 0) return;
        ProfScope ps(prof ? kPhase2 : -1, 2.0 * bs3 * (ld / BS - 1), s);
        enq((phase2_kernel<Ar, Alt, BS, P2W, TT>), dim3(2 * nt2),
                           dim3((BS / TT) * (P2W / TT)), s, X, ld, (int64_t)r * BS, nt2, ar, alt, mode,
                           skip);
    };
    auto p3_part = [&](int r, int set, hipStream_t st, int64_t seq0, int64_t seq_end) {
        const int64_t tiles = seq_end - seq0;
        if (tiles <= 0) return;
        const int per_xcd = (int)((tiles + 7) / 8);
        ProfScope ps(!prof ? -1 : set == kCross ? kPhase3Cross : kPhase3, (double)tiles * MT * MT * BS, st);
        const dim3 grid(8 * per_xcd), block((MT / TT) * (MT / TT));
        const int a = (int)seq0, b = (int)seq_end;
        if (set == kAll)
            enq((phase3_kernel<Ar, Alt, BS, MT, kAll, TT>), grid, block, st, X, ld, r,
                               per_xcd, a, b, ar, alt, mode, skip);
        else if (set == kRest)
            enq((phase3_kernel<Ar, Alt, BS, MT, kRest, TT>), grid, block, st, X, ld, r,
                               per_xcd, a, b, ar, alt, mode, skip);
        else
            enq((phase3_kernel<Ar, Alt, BS, MT, kCross, TT>), grid, block, st, X, ld, r,
                               per_xcd, a, b, ar, alt, mode, skip);
    };
    auto p3 = [&](int r, int set, hipStream_t st) { p3_part(r, set, st, 0, p3_count(set, nt, pb)); };
    // kRest in kRestChunks launches (one with the blocked phase 1 or the
    // closure): between them the caller stream's critical-path kernels find
    // free compute units
    // (one launch where phase 1 is the blocked closure: it fits in a slot a
    // kRest workgroup frees, so no launch boundary is needed to let it in,
    // and one launch has one tail instead of two; measured at n = 32768:
    // kRest 6.58 ms per round in one launch against 2 x 3.37 ms)
    auto p3_rest = [&](int r, hipStream_t st) {
        const int64_t total = p3_count(kRest, nt, pb);
        const int C = (blocked_p1 || closure) ? 1 : kRestChunks;  // (closure: n = 8192 17.0 -> 15.8 ms)
        for (int c = 0; c < C; ++c) p3_part(r, kRest, st, total * c / C, total * (c + 1) / C);
    };
    if (!aux) {
        for (int r = 0; r < R; ++r) {
            round_mark();
            p1(r);
            p2(r);
            p3(r, kAll, s);
        }
    } else {
        round_mark();
        p1(0);
        p2(0);
        APSP_HIP(enq_record(aux->panels, s));
        for (int r = 0; r + 1 < R; ++r) {
            if (r > 0) round_mark();
            APSP_HIP(enq_wait(aux->s, aux->panels));
            p3_rest(r, aux->s);
            if (r > 0) APSP_HIP(enq_wait(s, aux->rest));
            APSP_HIP(enq_record(aux->rest, aux->s));
            p3(r, kCross, s);
            p1(r + 1);
            p2(r + 1);
            APSP_HIP(enq_record(aux->panels, s));
        }
        APSP_HIP(enq_wait(s, aux->rest));
        p3(R - 1, kAll, s);
    }
    APSP_HIP(hipGetLastError());
    return APSP_SUCCESS;
}

// Kernel configurations: (block size, thread tile).  Thread tile 4 is the
// latency configuration for small n (64-wide blocks only).
template <class Ar, class Alt = NoAlt>
apsp_status_t run_rounds_bs(int bs, int tt, Sched sc, void *X, int64_t ld, const Ar &ar,
                            hipStream_t s, const int32_t *skip, const Alt &alt = Alt{},
                            const int32_t *mode = nullptr, bool prof = true) {
    if (tt == 4) {
        if (bs == 64) return run_rounds<Ar, Alt, 64, 4>(X, ld, ar, alt, mode, s, skip, sc, prof);
        return APSP_ERROR_INVALID_ARGUMENT;
    }
    switch (bs) {
        case 64: return run_rounds<Ar, Alt, 64, 8>(X, ld, ar, alt, mode, s, skip, sc, prof);
        case 128: return run_rounds<Ar, Alt, 128, 8>(X, ld, ar, alt, mode, s, skip, sc, prof);
        case 256:
            if constexpr (sizeof(typename Ar::T) == 4)
                return run_rounds<Ar, Alt, 256, 8>(X, ld, ar, alt, mode, s, skip, sc, prof);
            return APSP_ERROR_INVALID_ARGUMENT;
        default: return APSP_ERROR_INVALID_ARGUMENT;
    }
}

// Block size by n for distance rounds (measured on MI355X, int32
// distances in float32 arithmetic with the phase-1 closure, ms per solve
// for BS = 64 / 128 / 256): 4608: 5.09 / 5.95 / 5.40; 5120: 6.41 / 6.94 /
// 6.25; 5632: 7.90 / 7.95 / 7.40; 6144: 9.65 / 8.75 / 8.38; 6656: 11.62 /
// 9.72 / 9.24; 8192: 19.88 / 16.92 / 15.66; 12288: 66.1 / 52.3 / 48.4.
// With the closure, phase 1 of a 256-wide block no longer sets the pace,
// and the larger blocks' fewer rounds win from n of about 5000.  The
// fp64-key recurrence (the product route's fallback there) keeps BS = 128
// above n = 4096.
int auto_block(int64_t n, bool pred) {
    if (n <= 4096) return 64;
    if (pred) return 128;
    if (n <= 4864) return 64;
    return 256;
}

// The float32 predecessor route's distance rounds (measured with the
// closure, ms per solve at BS = 64 / 128 / 256, the key product included):
// 5120: 10.42 / 11.11 / 10.45; 6144: 15.65 / 14.94 / 14.77; 7168: 23.70 /
// 21.77 / 21.10; 8192: 33.08 / 30.55 / 29.48.
int auto_block_pp(int64_t n) {
    if (n <= 5888) return 64;
    if (n < 7168) return 128;
    return 256;
}

// 64-wide blocks take 4 x 4 register blocks (twice the workgroups of 8 x 8:
// at n = 4096, 4.30 vs 6.45 ms)
int auto_tile(int64_t, int bs) { return bs == 64 ? 4 : 8; }

// int32 distance solves run in float32 arithmetic (exact while watched,
// else redone in int32) when asked to, or automatically from n = 4096,
// where phase 3 dominates and the skipped int32 launches cost little
// (measured on MI355X: 4.08 vs 4.50 ms at n = 4096; slower at 3000 and below).
bool use_f32w(int64_t n, apsp_dtype_t dtype, bool with_pred, int arith) {
    if (dtype != APSP_INT32 || with_pred || arith == 1) return false;
    return arith == 2 || n >= 4096;
}

// Predecessor solves: float32 distances + the key product (exact, with
// the fp64-key recurrence as the device's fallback) when asked to, or
// automatically from n = 4096, where the product costs less than the
// recurrence's fp64 arithmetic (measured on MI355X, float32 / int32
// weights: 6.35 vs 7.06 / 6.29 vs 6.57 ms at n = 4096, 1.4x faster at 5120
// to 16384; even or slower at 3072 and below).
bool use_pp(int64_t n, bool with_pred, int arith) {
    if (!with_pred || arith == 1) return false;
    return arith == 2 || n >= 4096;
}

int pp_bits(int64_t n) {
    int S = 1;
    while ((int64_t(1) << S) < n) ++S;
    return S;
}

// Block sizes and padded orders of a predecessor solve with the product:
// the distance rounds (ld, a multiple of the 128-wide product tiles too)
// and the fallback recurrence (ldf <= ld).
struct PPShape {
    int bsd, bsf;
    int64_t ld, ldf;
};
PPShape pp_shape(int64_t n, int opt_bs) {
    PPShape p;
    p.bsd = opt_bs ? opt_bs : auto_block_pp(n);
    p.bsf = opt_bs ? std::min(opt_bs, 128) : auto_block(n, true);
    const int64_t m = std::max(p.bsd, 128);
    p.ld = (n + m - 1) / m * m;
    p.ldf = (n + p.bsf - 1) / p.bsf * p.bsf;
    return p;
}

// Work memory a solve needs beyond dist/pred (0 when it runs in place).
size_t work_bytes(int64_t n, bool with_pred, int opt_bs, bool aligned, apsp_dtype_t dtype, int arith) {
    if (use_pp(n, with_pred, arith)) {
        const int64_t ld = pp_shape(n, opt_bs).ld;
        return (size_t)(ld * ld) * 8 + 256;
    }
    const int bs = opt_bs ? opt_bs : auto_block(n, with_pred);
    const int64_t ld = (n + bs - 1) / bs * bs;
    if (with_pred) return (size_t)(ld * ld) * 8 + 256;
    if (use_f32w(n, dtype, with_pred, arith)) return (size_t)(ld * ld) * 4 + 256;
    if (ld == n && aligned) return 0;
    return (size_t)(ld * ld) * 4;
}

// Single-launch schedule: distances only, 64-wide blocks with 4 x 4 thread
// tiles, 4-byte arithmetic without a watch (int32 in int32, float32),
// issued directly or into a hipGraph (not while a stepper records, nor into
// caller-provided or static work memory); automatic up to a padded order of
// kSingleMaxLd.  One ordinary launch of flow_tasks_kernel over the whole
// matrix: int32 up to a padded order of 768 in 32-wide blocks (twice the
// rounds of 64-wide ones, each round's chain much shorter; above that the
// task count makes the shared task counter the bottleneck), else 64-wide
// blocks -- float32 always, the blocking of the per-phase launches, so the
// rounding is theirs too.  (Measured on MI355X, int32 distances, ms per
// solve, per-phase launches / 32-wide tasks / 64-wide tasks: n = 256 0.111
// / 0.082 / 0.107; 512 0.217 / 0.155 / 0.204; 1024 0.440 / 0.465 / 0.398;
// 2048 1.180 / 3.03 / 0.838; 3072 2.45 / - / 1.78; 4032 4.43 / - / 3.46.)
constexpr int64_t kSingleMaxLd = 4096;

inline bool single_applies(int64_t ld, int bs, int tt, bool with_pred, bool f32w, int schedule, bool ext_ws) {
    if (with_pred || f32w || bs != kSingleBS || tt != 4 || ext_ws || t_rec || t_noalloc) return false;
    return schedule == 3 || (schedule == 0 && ld <= kSingleMaxLd);
}

// The single launch's shape for padded order ld.
struct SinglePlan {
    int bs = 0;             // 32 or 64
    int groups = 0;         // workgroups taking tasks
    size_t word_bytes = 0;  // task words
    size_t pub_bytes = 0;   // the two publication matrices
};
#ifndef APSP_TASK32_MAX_LD
#define APSP_TASK32_MAX_LD 768
#endif
template <class Ar>
SinglePlan single_plan(int cus, int64_t ld) {
    SinglePlan p;
    p.bs = std::is_same_v<Ar, ArI32> && ld <= APSP_TASK32_MAX_LD ? 32 : 64;
    const int64_t R = ld / p.bs, m = R - 1;
    // workgroups: one per task of a round's phase 3, at most 4 per CU
    p.groups = (int)std::max<int64_t>(1, std::min<int64_t>(m * m, 4 * (int64_t)cus));
    p.word_bytes = task_word_bytes((int)R);
    p.pub_bytes = 2 * (size_t)(ld * ld) * 4;
    return p;
}

template <class Ar>
void run_single(void *X, int64_t ld, const Ar &ar, const SinglePlan &plan, void *ws, int32_t *status,
                const int32_t *skip, hipStream_t s) {
    ProfScope ps(kSingle, (double)ld * (double)ld * (double)ld, s);
    uint32_t *words = (uint32_t *)((char *)ws + plan.pub_bytes);
    void *prow = ws, *pcol = (char *)ws + plan.pub_bytes / 2;
    if constexpr (std::is_same_v<Ar, ArI32>) {
        if (plan.bs == 32) {
            enq((flow_tasks_kernel<Ar, 32>), dim3(plan.groups), dim3(kSingleThreads), s, X, ld, ld, ar, words, prow,
                pcol, status, skip);
            return;
        }
    }
    enq((flow_tasks_kernel<Ar, 64>), dim3(plan.groups), dim3(kSingleThreads), s, X, ld, ld, ar, words, prow, pcol,
        status, skip);
}

// Work memory of a single-launch solve (0 if the options do not take one):
// made before a graph capture, which cannot allocate.
size_t single_work_bytes(int64_t n, apsp_dtype_t dtype, bool with_pred, bool aligned, const apsp_options_t &opt) {
    const int bs = opt.block_size ? opt.block_size : auto_block(n, with_pred);
    const int tt = opt.thread_tile ? opt.thread_tile : auto_tile(n, bs);
    const int64_t ld = (n + bs - 1) / bs * bs;
    if (!single_applies(ld, bs, tt, with_pred, dtype == APSP_INT32 && opt.arith == 2, opt.schedule, false)) return 0;
    const SinglePlan p = dtype == APSP_INT32 ? single_plan<ArI32>(256, ld) : single_plan<ArF32>(256, ld);
    const size_t mat = (ld == n && aligned) ? 0 : (size_t)(ld * ld) * 4;
    return mat + p.pub_bytes + p.word_bytes;
}

template <class T>
apsp_status_t solve_typed(T *dist, int32_t *pred, int64_t n, hipStream_t s,
                          const apsp_options_t &opt, void *ext_ws, size_t ext_bytes) {
    int dev = 0;
    APSP_HIP(hipGetDevice(&dev));
    const bool with_pred = pred != nullptr;
    const int bs = opt.block_size ? opt.block_size : auto_block(n, with_pred);
    const int tt = opt.thread_tile ? opt.thread_tile : auto_tile(n, bs);
    if (tt == 4 && bs != 64) return APSP_ERROR_INVALID_ARGUMENT;
    const Sched lookahead{opt.schedule, opt.phase1};
    // device-gated fallback passes run their rounds in order
    const Sched in_order{1, opt.phase1};
    // caller-provided work memory (the server) or the per-stream cache
    auto workspace = [&](int d, hipStream_t st, size_t bytes, void **out) -> apsp_status_t {
        if (ext_ws) {
            if (ext_bytes < bytes) return APSP_ERROR_INVALID_ARGUMENT;
            *out = ext_ws;
            return APSP_SUCCESS;
        }
        return cached_workspace(d, st, bytes, out);
    };
    if (with_pred && bs == 256 && !use_pp(n, true, opt.arith)) return APSP_ERROR_INVALID_ARGUMENT;
    const int64_t ld = (n + bs - 1) / bs * bs;
    int32_t *status = opt.d_status;
    t_status = status;
    const int32_t *skip = nullptr;
    // the single launch (int32 in int32 arithmetic) where it applies, before
    // the automatic float32 route for int32 (at n = 4096 both apply: 3.5
    // against 4.2 ms)
    using ArPlain = std::conditional_t<std::is_same_v<T, int32_t>, ArI32, ArF32>;
    const bool single = single_applies(ld, bs, tt, with_pred, std::is_same_v<T, int32_t> && opt.arith == 2,
                                       opt.schedule, ext_ws != nullptr);
    const bool f32w = !single && std::is_same_v<T, int32_t> && use_f32w(n, APSP_INT32, with_pred, opt.arith);
    SinglePlan plan;
    if (single) {
        int cus = 0;
        APSP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        plan = single_plan<ArPlain>(cus, ld);
    }
    // single-launch schedule: [work matrix if padded][publication matrices][task words]
    void *single_ws = nullptr, *single_aux = nullptr;
    const size_t single_mat = (ld == n && (uintptr_t)dist % 16 == 0) ? 0 : (size_t)(ld * ld) * sizeof(T);
    if (single) {
        apsp_status_t st = workspace(dev, s, single_mat + plan.pub_bytes + plan.word_bytes, &single_ws);
        if (st != APSP_SUCCESS) return st;
        single_aux = (char *)single_ws + single_mat;
        // (the work memory is shared with other solves on this stream: its words are cleared per solve)
        uint32_t *words = (uint32_t *)((char *)single_aux + plan.pub_bytes);
        const int count = (int)(plan.word_bytes / 4);
        enq(flow_init_kernel, dim3(std::min(64, (count + 255) / 256)), dim3(256), s, words, count, status);
    } else if (status) {
        enq(status_init_kernel, dim3(1), dim3(1), s, status);
    }
    if (opt.validate) {
        enq((validate_kernel<T>), dim3(grid_for(n * n)), dim3(256), s, dist, n,
                           apsp_weight_bound(n), status);
        skip = status;
    }
    constexpr T inf = std::is_same_v<T, int32_t> ? T(kInf32) : T(__builtin_huge_valf());
    if (!f32w && opt.d_arith) enq(store_word_kernel, dim3(1), dim3(1), s, opt.d_arith, 0);
    if constexpr (std::is_same_v<T, int32_t>) {
        if (f32w) {
            // float32 pass (exact while watched), then an int32 pass that the
            // device runs only if a watcher fired; both use one work buffer
            const size_t mat = (size_t)(ld * ld) * 4;
            void *w = nullptr;
            apsp_status_t st = workspace(dev, s, mat + 256, &w);
            if (st != APSP_SUCCESS) return st;
            float *Xf = (float *)w;
            int32_t *words = (int32_t *)((char *)w + mat);
            enq(f32w_init_kernel, dim3(1), dim3(1), s, words);
            const int vec = (n % 4 == 0) && ((uintptr_t)dist % 16 == 0);
            enq(f32w_in_kernel, grid_rows(ld, ld), dim3(256), s, dist, n, Xf, ld, words, skip,
                               vec);
            ArF32W arw;
            arw.big = words;
            st = run_rounds_bs<ArF32W>(bs, tt, lookahead, Xf, ld, arw, s, skip);
            if (st != APSP_SUCCESS) return st;
            enq(f32w_out_kernel, grid_rows(n, n), dim3(256), s, Xf, ld, dist, n, status, words,
                               skip, vec);
            enq(f32w_gate_kernel, dim3(1), dim3(1), s, words, skip, opt.d_arith);
            const int32_t *gate = words + 1;
            int32_t *Xi = dist;
            if (!((ld == n) && ((uintptr_t)dist % 16 == 0))) {
                Xi = (int32_t *)w;  // the float32 matrix is no longer needed
                enq((pad_in_kernel<int32_t>), dim3(grid_for(ld * ld)), dim3(256), s, dist, n,
                                   Xi, ld, kInf32, gate);
            }
            // in order (3 launches per round): when the gate stays closed,
            // every launch still costs its dispatch
            st = run_rounds_bs<ArI32>(bs, tt, in_order, Xi, ld, ArI32{}, s, gate, NoAlt{}, nullptr, false);
            if (st != APSP_SUCCESS) return st;
            enq((finalize_kernel<int32_t>), dim3(grid_for(n * n)), dim3(256), s, Xi, ld, dist,
                               n, status, gate);
            APSP_HIP(hipGetLastError());
            return APSP_SUCCESS;
        }
    }
    if (use_pp(n, with_pred, opt.arith)) {
        // [X: ld^2 float32][B: ld^2 float32][words]; the fallback's fp64 keys
        // (ldf^2 x 8 bytes) reuse the two matrices
        const PPShape sh = pp_shape(n, opt.block_size);
        const int ttd = opt.thread_tile ? opt.thread_tile : auto_tile(n, sh.bsd);
        const int ttf = opt.thread_tile ? opt.thread_tile : auto_tile(n, sh.bsf);
        const size_t mat = (size_t)(sh.ld * sh.ld) * 4;
        void *w = nullptr;
        apsp_status_t st = workspace(dev, s, 2 * mat + 256, &w);
        if (st != APSP_SUCCESS) return st;
        float *X = (float *)w;
        float *Bm = (float *)((char *)w + mat);
        int32_t *words = (int32_t *)((char *)w + 2 * mat);
        const int S = pp_bits(n);
        const int vec = (n % 4 == 0) && ((uintptr_t)dist % 16 == 0);
        enq(pp_init_kernel, dim3(1), dim3(1), s, words);
        enq((pp_in_kernel<T>), grid_rows(sh.ld, sh.ld), dim3(256), s, dist, n, X, Bm, sh.ld, S,
                           (float)apsp_weight_bound(n), words, skip, vec);
        enq(pp_rounds_gate_kernel, dim3(1), dim3(1), s, words, skip);
        ArF32W arw;
        arw.big = words + kPPBig;
        st = run_rounds_bs<ArF32W>(sh.bsd, ttd, lookahead, X, sh.ld, arw, s, words + kPPRounds);
        if (st != APSP_SUCCESS) return st;
        enq((pp_out_kernel<T>), grid_rows(n, n), dim3(256), s, X, sh.ld, dist, n, S, words,
                           status, skip, vec);
        enq(pp_product_gate_kernel, dim3(1), dim3(1), s, words);
        {
            const int nt = (int)((n + 127) / 128);
            const int per_xcd = (nt * nt + 7) / 8;
            const int kcount = (int)((n + 31) / 32 * 32);
            ProfScope ps(kPredProduct, (double)n * (double)n * (double)kcount, s);
            enq((pp_product_kernel<T>), dim3(8 * per_xcd), dim3(256), s, X, Bm, sh.ld, kcount,
                               dist, pred, n, S, nt, per_xcd, words, skip);
        }
        enq(pp_gate_kernel, dim3(1), dim3(1), s, words, skip, opt.d_arith);
        const int32_t *gate = words + kPPGate;
        enq((pp_restore_kernel<T>), dim3(grid_for(n * n)), dim3(256), s, Bm, sh.ld, dist, n, S,
                           words);
        // the fallback: the exact fp64-key recurrence (pairs for float32
        // weights that are not integers within the bound)
        int32_t *mode = std::is_same_v<T, float> ? words + kPPMode : nullptr;
        ArKey ar{pred_bits(sh.ldf)};
        enq((pred_pack_kernel<T>), dim3(grid_for(sh.ldf * sh.ldf)), dim3(256), s, dist, n, w,
                           sh.ldf, ar.S, mode, gate);
        // in order (3 launches per round), as a closed gate still costs
        // every launch's dispatch
        if constexpr (std::is_same_v<T, float>)
            st = run_rounds_bs<ArKey, ArLexF32>(sh.bsf, ttf, in_order, w, sh.ldf, ar, s, gate, ArLexF32{}, mode, false);
        else
            st = run_rounds_bs<ArKey>(sh.bsf, ttf, in_order, w, sh.ldf, ar, s, gate, NoAlt{}, nullptr, false);
        if (st != APSP_SUCCESS) return st;
        enq((pred_unpack_kernel<T>), dim3(grid_for(n * n)), dim3(256), s, w, sh.ldf, dist, pred,
                           n, ar.S, mode, status, gate);
        APSP_HIP(hipGetLastError());
        return APSP_SUCCESS;
    }
    if (!with_pred) {
        T *X = dist;
        const bool inplace = (ld == n) && ((uintptr_t)dist % 16 == 0);
        if (!inplace) {
            void *w = single_ws;
            if (!single) {
                apsp_status_t st = workspace(dev, s, (size_t)(ld * ld) * sizeof(T), &w);
                if (st != APSP_SUCCESS) return st;
            }
            X = (T *)w;
            enq((pad_in_kernel<T>), dim3(grid_for(ld * ld)), dim3(256), s, dist, n, X,
                               ld, inf, skip);
        }
        apsp_status_t st;
        if (single) {
            run_single<ArPlain>(X, ld, ArPlain{}, plan, single_aux, status, skip, s);
            st = APSP_SUCCESS;
        } else
            st = run_rounds_bs<ArPlain>(bs, tt, lookahead, X, ld, ArPlain{}, s, skip);
        if (st != APSP_SUCCESS) return st;
        // (a failed single-launch wait leaves APSP_ERROR_TIMEOUT in status: no wrap-up then)
        const int32_t *fskip = single && status ? (const int32_t *)status : skip;
        if constexpr (std::is_same_v<T, float>) {
            if (X == dist) {
                enq(finalize_diag_kernel, dim3((unsigned)std::min<int64_t>(64, (n + 255) / 256)), dim3(256), s,
                    (const float *)X, ld, n, status, fskip);
                APSP_HIP(hipGetLastError());
                return APSP_SUCCESS;
            }
        }
        enq((finalize_kernel<T>), dim3(grid_for(n * n)), dim3(256), s, X, ld, dist, n, status, fskip);
    } else {
        // ld^2 8-byte elements, then one int32 mode word
        void *w = nullptr;
        const size_t mat = (size_t)(ld * ld) * 8;
        apsp_status_t st = workspace(dev, s, mat + 256, &w);
        if (st != APSP_SUCCESS) return st;
        int32_t *mode = nullptr;
        ArKey ar{pred_bits(ld)};
        if constexpr (std::is_same_v<T, float>) {
            mode = (int32_t *)((char *)w + mat);
            enq(mode_init_kernel, dim3(1), dim3(1), s, mode);
            enq(integral_check_kernel, dim3(grid_for(n * n)), dim3(256), s, dist, n,
                               (float)apsp_weight_bound(n), mode);
        }
        enq((pred_pack_kernel<T>), dim3(grid_for(ld * ld)), dim3(256), s, dist, n, w,
                           ld, ar.S, mode, skip);
        if constexpr (std::is_same_v<T, float>)
            st = run_rounds_bs<ArKey, ArLexF32>(bs, tt, lookahead, w, ld, ar, s, skip, ArLexF32{}, mode);
        else
            st = run_rounds_bs<ArKey>(bs, tt, lookahead, w, ld, ar, s, skip);
        if (st != APSP_SUCCESS) return st;
        enq((pred_unpack_kernel<T>), dim3(grid_for(n * n)), dim3(256), s, w, ld, dist,
                           pred, n, ar.S, mode, status, skip);
    }
    APSP_HIP(hipGetLastError());
    return APSP_SUCCESS;
}

}  // namespace

// Closure scratch a stepper or a lent work area must carry (the rounds of
// 128- or 256-wide blocks take the dataflow closure; a predecessor solve's
// distance rounds take the distance block size).
size_t closure_bytes(int64_t n, bool with_pred, int opt_bs) {
    const int bs = opt_bs ? opt_bs : std::max(auto_block(n, with_pred), auto_block(n, false));
    return bs >= 128 ? kClosureBytes : 0;
}

size_t solve_work_bytes(int64_t n, apsp_dtype_t dtype, bool with_pred) {
    return work_bytes(n, with_pred, 0, true, dtype, 0) + closure_bytes(n, with_pred, 0);
}

namespace {

apsp_status_t solve_direct(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype, hipStream_t s,
                           const apsp_options_t &opt_in, void *ws, size_t ws_bytes) {
    apsp_options_t opt = opt_in;
    if (opt.schedule == 3) {  // the single-launch schedule's one configuration
        opt.block_size = 64;
        opt.thread_tile = 4;
        if (dtype == APSP_INT32) opt.arith = 1;
    }
    if (dtype == APSP_INT32) return solve_typed<int32_t>((int32_t *)dist, pred, n, s, opt, ws, ws_bytes);
    return solve_typed<float>((float *)dist, pred, n, s, opt, ws, ws_bytes);
}

// hipGraph cache (apsp_options_t.use_graph): one executable graph per
// (device, stream, shape, options, buffer addresses), replayed instead of
// re-issuing the launch sequence.
struct GraphKey {
    int dev;
    hipStream_t s;
    int64_t n;
    int dtype, validate, bs, tt, schedule, arith, phase1;
    void *dist, *pred, *status, *ws, *arith_used;
    bool operator<(const GraphKey &o) const {
        return std::tie(dev, s, n, dtype, validate, bs, tt, schedule, arith, phase1, dist, pred, status, ws,
                        arith_used) < std::tie(o.dev, o.s, o.n, o.dtype, o.validate, o.bs, o.tt, o.schedule,
                                               o.arith, o.phase1, o.dist, o.pred, o.status, o.ws, o.arith_used);
    }
};
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;
constexpr size_t kMaxGraphs = 64;

void drop_graphs_locked(int dev) {
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        if (dev < 0 || it->first.dev == dev) {
            (void)hipGraphExecDestroy(it->second);
            it = g_graphs.erase(it);
        } else {
            ++it;
        }
    }
}

apsp_status_t solve_graph(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype, hipStream_t s,
                          const apsp_options_t &opt, void *ws, size_t ws_bytes) {
    int dev = 0;
    APSP_HIP(hipGetDevice(&dev));
    const bool with_pred = pred != nullptr;
    const int bs = opt.block_size ? opt.block_size : auto_block(n, with_pred);
    const int tt = opt.thread_tile ? opt.thread_tile : auto_tile(n, bs);
    // the work memory must exist (at its final address) before recording
    void *w = ws;
    const bool aligned = ((uintptr_t)dist % 16) == 0;
    size_t need = work_bytes(n, with_pred, opt.block_size, aligned, dtype, opt.arith);
    if (!ws) {
        apsp_options_t o = opt;  // the single launch's configuration, as solve_direct sets it
        if (o.schedule == 3) {
            o.block_size = 64;
            o.thread_tile = 4;
            if (dtype == APSP_INT32) o.arith = 1;
        }
        need = std::max(need, single_work_bytes(n, dtype, with_pred, aligned, o));
    }
    if (!w && need > 0) {
        apsp_status_t st = cached_workspace(dev, s, need, &w);
        if (st != APSP_SUCCESS) return st;
    }
    if (opt.schedule != 1) {  // create the auxiliary stream outside the recording
        AuxStream *aux = nullptr;
        apsp_status_t st = aux_stream(dev, s, &aux);
        if (st != APSP_SUCCESS) return st;
    }
    if ((opt.phase1 == 0 || opt.phase1 == 3) && closure_bytes(n, with_pred, opt.block_size) > 0) {
        // and the phase-1 closure's scratch
        void *c = nullptr;
        apsp_status_t st = closure_scratch(dev, s, true, &c);
        if (st != APSP_SUCCESS) return st;
    }
    GraphKey key{dev,  s,    n,    (int)dtype,   opt.validate, bs, tt, opt.schedule, opt.arith, opt.phase1,
                 dist, pred, opt.d_status, w, opt.d_arith};
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        if (g_graphs.size() >= kMaxGraphs) drop_graphs_locked(-1);
        APSP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        t_capturing = true;
        apsp_status_t st = solve_direct(dist, pred, n, dtype, s, opt, ws, ws_bytes);
        t_capturing = false;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (st != APSP_SUCCESS) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            return APSP_ERROR_HIP;
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            return APSP_ERROR_HIP;
        }
        it = g_graphs.emplace(key, exec).first;
    }
    APSP_HIP(hipGraphLaunch(it->second, s));
    return APSP_SUCCESS;
}

}  // namespace

// Host-side checks shared by apsp_solve_ex and the steppers.
apsp_status_t check_options(int64_t n, apsp_dtype_t dtype, bool with_pred, const apsp_options_t &opt) {
    if (n < 0 || n > kMaxN) return APSP_ERROR_INVALID_ARGUMENT;
    if (dtype != APSP_INT32 && dtype != APSP_FLOAT32) return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.block_size != 0 && opt.block_size != 64 && opt.block_size != 128 && opt.block_size != 256)
        return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.thread_tile != 0 && opt.thread_tile != 4 && opt.thread_tile != 8) return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.thread_tile == 4 && opt.block_size != 0 && opt.block_size != 64) return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.arith < 0 || opt.arith > 2) return APSP_ERROR_INVALID_ARGUMENT;
    // 256-wide blocks hold 4-byte elements only: with predecessors they serve
    // the distance rounds of the float32 route (its fallback recurrence
    // takes 128-wide blocks)
    if (opt.block_size == 256 && with_pred && !use_pp(n, true, opt.arith)) return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.validate && !opt.d_status) return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.schedule < 0 || opt.schedule > 3) return APSP_ERROR_INVALID_ARGUMENT;
    // the single-launch schedule: distances on 64-wide blocks with 4 x 4 thread
    // tiles, int32 weights in int32 arithmetic
    if (opt.schedule == 3 &&
        (with_pred || n > kSingleMaxN || (opt.block_size != 0 && opt.block_size != 64) ||
         (opt.thread_tile != 0 && opt.thread_tile != 4) || (dtype == APSP_INT32 && opt.arith == 2)))
        return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.phase1 < 0 || opt.phase1 > 3) return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.phase1 == 2 && opt.block_size != 256) return APSP_ERROR_INVALID_ARGUMENT;
    if (opt.phase1 == 3 && opt.block_size != 128 && opt.block_size != 256) return APSP_ERROR_INVALID_ARGUMENT;
    return APSP_SUCCESS;
}

// Static work memory of apsp_solve_noalloc: the largest work matrix any
// solve of n <= 2048 needs (2048^2 8-byte keys, or two 2048^2 float32
// matrices, plus the route's status words), then the phase-1 closure's
// scratch (zero from load; each closure launch leaves its words zeroed).
// One copy per device, held until the process ends; in host code the name
// only stands for the symbol, so kernels get the device address found by
// hipGetSymbolAddress.
constexpr size_t kScratchWork = (size_t)2048 * 2048 * 8 + 4096;
constexpr size_t kScratchBytes = kScratchWork + kClosureBytes;  // [work][closure scratch]
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// The calling device's copy of scratch (looked up once per device).
apsp_status_t scratch_ptr(void **out) {
    int dev = 0;
    APSP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return APSP_ERROR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        APSP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return APSP_ERROR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return APSP_SUCCESS;
}

apsp_status_t solve_internal(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype, hipStream_t s,
                             const apsp_options_t &opt, void *ws, size_t ws_bytes) {
    if (n == 0) return APSP_SUCCESS;
    // graphs cannot be recorded on the legacy default stream
    if (opt.use_graph && s != nullptr) return solve_graph(dist, pred, n, dtype, s, opt, ws, ws_bytes);
    return solve_direct(dist, pred, n, dtype, s, opt, ws, ws_bytes);
}

}  // namespace apsp

using namespace apsp;

extern "C" {

const char *apsp_status_string(apsp_status_t st) {
    switch (st) {
        case APSP_SUCCESS: return "success";
        case APSP_ERROR_INVALID_ARGUMENT: return "invalid argument";
        case APSP_ERROR_INVALID_VALUE: return "invalid value";
        case APSP_ERROR_NEGATIVE_CYCLE: return "negative cycle";
        case APSP_ERROR_OUT_OF_MEMORY: return "out of memory";
        case APSP_ERROR_HIP: return "HIP runtime error";
        case APSP_ERROR_QUEUE_FULL: return "queue full";
        case APSP_ERROR_NOT_READY: return "not ready";
        case APSP_ERROR_CANCELLED: return "cancelled";
        case APSP_ERROR_TIMEOUT: return "timeout";
        case APSP_ERROR_UNKNOWN_TICKET: return "unknown ticket";
    }
    return "unknown status";
}

int apsp_last_hip_error(void) { return g_last_hip; }

int apsp_version(void) { return 100; }

int64_t apsp_weight_bound(int64_t n) { return weight_bound(n); }

apsp_status_t apsp_solve_ex(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype,
                            hipStream_t stream, const apsp_options_t *options) {
    apsp_options_t opt{};
    if (options) opt = *options;
    const apsp_status_t bad = check_options(n, dtype, pred != nullptr, opt);
    if (bad != APSP_SUCCESS) return bad;
    if (n == 0) return APSP_SUCCESS;
    if (!dist || ((uintptr_t)dist % 4) != 0 || ((uintptr_t)pred % 4) != 0)
        return APSP_ERROR_INVALID_ARGUMENT;
    return solve_internal(dist, pred, n, dtype, stream, opt, nullptr, 0);
}

apsp_status_t apsp_solve(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype, hipStream_t stream) {
    return apsp_solve_ex(dist, pred, n, dtype, stream, nullptr);
}

int64_t apsp_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

apsp_status_t apsp_solve_noalloc(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype, hipStream_t stream,
                                 const apsp_options_t *options) {
    apsp_options_t opt{};
    if (options) opt = *options;
    const apsp_status_t bad = check_options(n, dtype, pred != nullptr, opt);
    if (bad != APSP_SUCCESS) return bad;
    // rounds in order on the caller's stream: the two-stream split would need a
    // second stream and events, a hipGraph an instantiation
    if (opt.use_graph || opt.schedule >= 2) return APSP_ERROR_INVALID_ARGUMENT;
    opt.schedule = 1;
    if (n == 0) return APSP_SUCCESS;
    if (!dist || ((uintptr_t)dist % 4) != 0 || ((uintptr_t)pred % 4) != 0) return APSP_ERROR_INVALID_ARGUMENT;
    const size_t need =
        work_bytes(n, pred != nullptr, opt.block_size, ((uintptr_t)dist % 16) == 0, dtype, opt.arith);
    if (need > kScratchWork) return APSP_ERROR_INVALID_ARGUMENT;  // beyond the static scratch
    void *ws = nullptr;
    {
        const apsp_status_t st = scratch_ptr(&ws);
        if (st != APSP_SUCCESS) return st;
    }
    t_noalloc = true;
    t_closure = (char *)ws + kScratchWork;
    const apsp_status_t st = solve_direct(dist, pred, n, dtype, stream, opt, need > 0 ? ws : nullptr, kScratchWork);
    t_closure = nullptr;
    t_noalloc = false;
    return st;
}

apsp_status_t apsp_profile_begin(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof.clear();
    g_prof_on = true;
    return APSP_SUCCESS;
}

apsp_status_t apsp_profile_end(apsp_profile_t *out) {
    if (!out) return APSP_ERROR_INVALID_ARGUMENT;
    std::vector<ProfRecord> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_on = false;
        recs.swap(g_prof);
    }
    *out = apsp_profile_t{};
    apsp_kernel_time_t *slot[9] = {&out->phase1,         &out->phase2,        &out->phase3,
                                   &out->other,          &out->phase3_cross,  &out->pred_product,
                                   &out->phase1_blocked, &out->single_launch, &out->phase1_flow};
    apsp_status_t st = APSP_SUCCESS;
    for (auto &r : recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            st = APSP_ERROR_HIP;
        }
        for (int kind : {r.kind == kPhase1Blocked || r.kind == kPhase1Flow ? (int)kPhase1 : -1, r.kind}) {
            if (kind < 0) continue;
            apsp_kernel_time_t *k = slot[kind];
            k->launches += 1;
            k->total_ms += ms;
            k->max_ms = std::max(k->max_ms, (double)ms);
            k->updates += r.updates;
        }
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    return st;
}

}  // extern "C"

// A recorded solve issued in slices of rounds (round-level preemption): it
// owns its work memory and second stream, so its slices may interleave with
// any other work, including other steppers on the same caller stream.
struct apsp_stepper {
    int device = 0;
    int64_t n = 0;
    apsp_dtype_t dtype = APSP_INT32;
    bool want_pred = false;
    apsp_options_t opt{};
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool owns_ws = true;  // false: work memory lent by the server
    size_t closure_bytes = 0;  // closure scratch at the end of ws
    AuxStream aux{};
    Recorder rec;
    hipStream_t stream = nullptr;
    size_t next = 0;  // next operation to issue
    bool begun = false;
};

namespace {

struct RecordScope {
    RecordScope(Recorder *r, AuxStream *a, void *closure) {
        t_rec = r;
        t_aux = a;
        t_closure = closure;
    }
    ~RecordScope() {
        t_rec = nullptr;
        t_aux = nullptr;
        t_closure = nullptr;
    }
};


}  // namespace

extern "C" {

}  // extern "C"

namespace apsp {

// lend == false: the stepper allocates (and frees) work memory for any
// alignment of dist; lend == true: it uses the caller's ws_bytes at ws (null
// when 0), which must cover a solve of (n, pred, options) on a 16-byte
// aligned dist (begin fails with APSP_ERROR_INVALID_ARGUMENT otherwise).
apsp_status_t stepper_create(int64_t n, apsp_dtype_t dtype, bool want_pred, const apsp_options_t *options,
                             bool lend, void *ws, size_t ws_bytes, apsp_stepper_t **out) {
    if (!out) return APSP_ERROR_INVALID_ARGUMENT;
    *out = nullptr;
    apsp_options_t opt{};
    if (options) opt = *options;
    opt.use_graph = 0;  // a stepper issues recorded operations itself
    apsp_status_t st = check_options(n, dtype, want_pred, opt);
    if (st != APSP_SUCCESS) return st;
    if (opt.schedule == 3) return APSP_ERROR_INVALID_ARGUMENT;  // one launch has no slices
    auto *p = new apsp_stepper();
    p->n = n;
    p->dtype = dtype;
    p->want_pred = want_pred;
    p->opt = opt;
    hipError_t e = hipGetDevice(&p->device);
    // work memory for any alignment of the caller's matrix
    // [work memory][closure scratch, if its rounds take the closure]
    p->closure_bytes = n ? closure_bytes(n, p->want_pred, opt.block_size) : 0;
    const size_t need = n ? work_bytes(n, p->want_pred, opt.block_size, lend, dtype, opt.arith) + p->closure_bytes : 0;
    if (lend) {
        if (ws_bytes < need) {
            delete p;
            return APSP_ERROR_INVALID_ARGUMENT;
        }
        p->ws = ws;
        p->ws_bytes = ws_bytes;
        p->owns_ws = false;
    } else {
        p->ws_bytes = need;
        if (e == hipSuccess && p->ws_bytes) e = hipMalloc(&p->ws, p->ws_bytes);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->aux.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->aux.panels, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->aux.rest, hipEventDisableTiming);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        stepper_destroy(p, true);
        return e == hipErrorOutOfMemory ? APSP_ERROR_OUT_OF_MEMORY : APSP_ERROR_HIP;
    }
    *out = p;
    return APSP_SUCCESS;
}

// sync: wait for the stepper's streams first (the server destroys steppers
// whose final event it has already seen complete, and must not block on the
// other work of a shared stream).
apsp_status_t stepper_destroy(apsp_stepper_t *p, bool sync) {
    if (!p) return APSP_ERROR_INVALID_ARGUMENT;
    bool ok = true;
    if (sync && p->begun) ok &= hipStreamSynchronize(p->stream) == hipSuccess;
    if (sync && p->aux.s) ok &= hipStreamSynchronize(p->aux.s) == hipSuccess;
    if (p->ws && p->owns_ws) ok &= hipFree(p->ws) == hipSuccess;
    if (p->aux.panels) (void)hipEventDestroy(p->aux.panels);
    if (p->aux.rest) (void)hipEventDestroy(p->aux.rest);
    if (p->aux.s) (void)hipStreamDestroy(p->aux.s);
    delete p;
    return ok ? APSP_SUCCESS : APSP_ERROR_HIP;
}

}  // namespace apsp

extern "C" {

apsp_status_t apsp_stepper_create(int64_t n, apsp_dtype_t dtype, int32_t want_pred, const apsp_options_t *options,
                                  apsp_stepper_t **out) {
    return stepper_create(n, dtype, want_pred != 0, options, false, nullptr, 0, out);
}

apsp_status_t apsp_stepper_begin(apsp_stepper_t *p, void *dist, int32_t *pred, hipStream_t stream) {
    if (!p) return APSP_ERROR_INVALID_ARGUMENT;
    if ((pred != nullptr) != p->want_pred) return APSP_ERROR_INVALID_ARGUMENT;
    if (p->n > 0 && (!dist || ((uintptr_t)dist % 4) != 0 || ((uintptr_t)pred % 4) != 0))
        return APSP_ERROR_INVALID_ARGUMENT;
    if (p->begun && p->next < p->rec.ops.size()) return APSP_ERROR_NOT_READY;  // the last solve is not issued
    p->rec.ops.clear();
    p->rec.marks.clear();
    p->next = 0;
    p->begun = false;
    if (p->n > 0) {
        int dev = 0;
        APSP_HIP(hipGetDevice(&dev));
        if (dev != p->device) return APSP_ERROR_INVALID_ARGUMENT;
        // [work memory][closure scratch]
        RecordScope rs(&p->rec, &p->aux,
                       p->closure_bytes ? (char *)p->ws + (p->ws_bytes - p->closure_bytes) : nullptr);
        apsp_status_t st =
            solve_direct(dist, pred, p->n, p->dtype, stream, p->opt, p->ws, p->ws_bytes - p->closure_bytes);
        if (st != APSP_SUCCESS) {
            p->rec.ops.clear();
            p->rec.marks.clear();
            return st;
        }
    }
    p->stream = stream;
    p->begun = true;
    return APSP_SUCCESS;
}

apsp_status_t apsp_stepper_step(apsp_stepper_t *p, int32_t rounds, int32_t *done) {
    if (!p || !p->begun) return APSP_ERROR_INVALID_ARGUMENT;
    const auto &ops = p->rec.ops;
    const auto &marks = p->rec.marks;
    size_t stop = ops.size();
    if (rounds > 0) {
        // rounds whose first operation is already issued, then `rounds` more
        const size_t started = (size_t)(std::lower_bound(marks.begin(), marks.end(), p->next) - marks.begin());
        if (started + (size_t)rounds < marks.size()) stop = marks[started + (size_t)rounds];
    }
    for (; p->next < stop; ++p->next) {
        const hipError_t e = ops[p->next]();
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            return APSP_ERROR_HIP;
        }
    }
    if (done) *done = p->next == ops.size() ? 1 : 0;
    return APSP_SUCCESS;
}

int64_t apsp_stepper_rounds(const apsp_stepper_t *p) { return p ? (int64_t)p->rec.marks.size() : -1; }

apsp_status_t apsp_stepper_destroy(apsp_stepper_t *p) { return stepper_destroy(p, true); }

apsp_status_t apsp_release_workspace(void) {
    int dev = 0;
    APSP_HIP(hipGetDevice(&dev));
    sweep_retired(true);
    APSP_HIP(hipDeviceSynchronize());
    {
        std::lock_guard<std::mutex> lg(g_graph_mu);
        drop_graphs_locked(dev);  // graphs refer to the work memory freed below
    }
    {
        std::lock_guard<std::mutex> la(g_aux_mu);
        for (auto it = g_aux.begin(); it != g_aux.end();) {
            if (it->first.first == dev) {
                aux_destroy(it->second);
                it = g_aux.erase(it);
            } else {
                ++it;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lc(g_closure_mu);
        for (auto it = g_closure.begin(); it != g_closure.end();) {
            if (it->first.first == dev) {
                if (it->second) APSP_HIP(hipFree(it->second));
                it = g_closure.erase(it);
            } else {
                ++it;
            }
        }
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.first == dev) {
            if (it->second.ptr) APSP_HIP(hipFree(it->second.ptr));
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
    return APSP_SUCCESS;
}

}  // extern "C"
