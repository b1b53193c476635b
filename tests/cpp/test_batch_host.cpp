// CPU test of the batched plans' host side and a bounds model of the
// batched kernels' indexing.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_cpp.py.
//
// 1. plan_args_check / batch_order / batch_meta_with (the code the plans
//    and the server run) over edge cases and thousands of seeded random
//    batches: the metadata image has the documented layout, the order is
//    largest first and stable, the work matrices fit the per-workgroup
//    scratch, the lean-kernel decision follows its rule.
// 2. For every graph of those batches, the index ranges the kernels compute
//    (restated here from the kernels' loop bounds and index formulas, not
//    shared with them): work-matrix tiles, panels and k-ranges of every
//    round in the lean kernel (both block widths) and the general kernel
//    (all three team configurations), and every LDS and global offset of
//    the tile routines for every tile shape the kernels instantiate,
//    including wavefront tiles with 8- and 16-element k-chunks, for every
//    thread of the workgroup.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "apsp_batch_host.h"

using namespace apsp;

static int g_failures = 0;
#define CHECK(cond)                                                                 \
    do {                                                                            \
        if (!(cond)) {                                                              \
            if (g_failures < 20) std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++g_failures;                                                           \
        }                                                                           \
    } while (0)

// ------------------------------------------------ tile routine LDS/global model
// LDS-DMA tile product (MT x NT C tile, KC-wide k-chunks, TM x TN per thread,
// 4-byte elements: VW = 4): checks every thread's copy destinations and
// sources and its compute reads against the buffers.
static void check_dma_shape(int MT, int NT, int KC, int TM, int TN) {
    const int VW = 4, TX = NT / TN, TY = MT / TM, NTH = TX * TY, NWAVES = NTH / 64;
    const int GN = TN / VW, GSTRIDE = NT / GN, KP = KC / VW;
    const int IA = MT * KC / VW / 64, IB = KC * NT / VW / 64;
    CHECK(NTH % 64 == 0 && GSTRIDE == TX * VW && (KP & (KP - 1)) == 0 && KP >= 2);
    CHECK(IA % NWAVES == 0 && IB % NWAVES == 0);
    auto swz = [&](int row) { return ((row * KP) >> 3) & (KP - 1); };
    for (int tid = 0; tid < NTH; ++tid) {
        const int lane = tid & 63, wave = tid >> 6;
        for (int j = 0; j < IA / NWAVES; ++j) {
            const int i = wave * (IA / NWAVES) + j, v = i * 64 + lane;
            const int row = v / KP, piece = v % KP;
            CHECK(row < MT && (piece ^ swz(row)) < KP);
            CHECK((i * 64 + lane) * VW + VW <= MT * KC);  // LDS destination of the 16 bytes
        }
        for (int j = 0; j < IB / NWAVES; ++j) {
            const int i = wave * (IB / NWAVES) + j, v = i * 64 + lane;
            const int row = v / (NT / VW), cv = v % (NT / VW);
            CHECK(row < KC && cv * VW + VW <= NT);
            CHECK((i * 64 + lane) * VW + VW <= KC * NT);
        }
        const int tx = tid % TX, ty = tid / TX;
        for (int kg = 0; kg < KC; kg += VW)
            for (int m = 0; m < TM; ++m) {
                const int row = ty + TY * m;
                CHECK(row < MT && row * KC + ((kg / VW) ^ swz(row)) * VW + VW <= MT * KC);
            }
        for (int kk = 0; kk < KC; ++kk)
            for (int g = 0; g < GN; ++g) CHECK(kk * NT + g * GSTRIDE + tx * VW + VW <= KC * NT);
        for (int m = 0; m < TM; ++m)
            for (int g = 0; g < GN; ++g) CHECK(ty + TY * m < MT && g * GSTRIDE + tx * VW + VW <= NT);  // C
    }
}

// Register-staged tile product (LDS rows padded by one vector), workgroup or
// wavefront (NTH = 64) form.
static void check_staged_shape(int MT, int NT, int KC, int TM, int TN, int VW) {
    const int TX = NT / TN, TY = MT / TM, NTH = TX * TY, GN = TN / VW, GSTRIDE = NT / GN;
    const int LDA = KC + VW, NA = MT * KC / VW, NB = KC * NT / VW;
    const int PA = (NA + NTH - 1) / NTH, PB = (NB + NTH - 1) / NTH;
    CHECK(TN % VW == 0 && GSTRIDE == TX * VW && KC % VW == 0);
    for (int tid = 0; tid < NTH; ++tid) {
        for (int i = 0; i < PA; ++i) {
            const int v = tid + NTH * i;
            if (v >= NA) continue;
            const int row = v / (KC / VW), cv = v % (KC / VW);
            CHECK(row < MT && cv * VW + VW <= KC);
            CHECK(row * LDA + cv * VW + VW <= MT * LDA);
        }
        for (int i = 0; i < PB; ++i) {
            const int v = tid + NTH * i;
            if (v >= NB) continue;
            const int row = v / (NT / VW), cv = v % (NT / VW);
            CHECK(row < KC && row * NT + cv * VW + VW <= KC * NT);
        }
        const int tx = tid % TX, ty = tid / TX;
        for (int kg = 0; kg < KC; kg += VW)
            for (int m = 0; m < TM; ++m) CHECK((ty + TY * m) * LDA + kg + VW <= MT * LDA);
        for (int kk = 0; kk < KC; ++kk)
            for (int g = 0; g < GN; ++g) CHECK(kk * NT + g * GSTRIDE + tx * VW + VW <= KC * NT);
    }
}

// Phase-1 register blocks: BS x BS block, TM1 x TN1 per thread; publications
// of 4 rows of BS elements per buffer.
static void check_phase1_shape(int BS, int TM1, int TN1, int VW) {
    const int TX = BS / TN1, TY = BS / TM1;
    for (int tid = 0; tid < TX * TY; ++tid) {
        const int tx = tid % TX, ty = tid / TX;
        CHECK(ty * TM1 + TM1 <= BS && tx * TN1 + TN1 <= BS);
        for (int g = 0; g < TM1 / VW; ++g) CHECK(ty * TM1 + g * VW + VW <= BS);
        for (int g = 0; g < TN1 / VW; ++g) CHECK(tx * TN1 + g * VW + VW <= BS);
    }
}

// ---------------------------------------------------------- round models
struct Tile {
    int64_t crow, ccol, h, w, k0, kc;
};

// A tile product on an ldp x ldp work matrix: C, A and B inside, k-range whole
// double chunks.
static void check_tile(const Tile &t, int64_t ldp, int chunk2) {
    CHECK(t.crow >= 0 && t.ccol >= 0 && t.crow + t.h <= ldp && t.ccol + t.w <= ldp);
    CHECK(t.k0 >= 0 && t.k0 + t.kc <= ldp && t.kc > 0 && t.kc % chunk2 == 0);
}

// The lean kernel's rounds for one graph (BMAX = 64 or 128).
static void model_lean(int64_t n, int BMAX, int64_t scratch_elems) {
    const int64_t ldp = (n + 63) / 64 * 64;
    CHECK(ldp * ldp <= scratch_elems);
    const int64_t R = (ldp + BMAX - 1) / BMAX;
    auto width = [&](int64_t q) { return std::min<int64_t>(BMAX, ldp - q * BMAX); };
    for (int64_t r = 0; r < R; ++r) {
        const int64_t r0 = r * BMAX, wr = width(r);
        CHECK(wr == 64 || wr == 128);
        const int64_t kc = r + 1 < R ? wr : std::min<int64_t>(wr, (n - r0 + 31) / 32 * 32);
        CHECK(n - r0 >= 1 && kc % 32 == 0 && kc >= 32 && kc <= wr);  // phase 1: ksteps whole 16s
        CHECK(r0 + wr <= ldp);
        for (int64_t q = 0; q < R; ++q) {
            if (q == r) continue;
            check_tile({r0, q * BMAX, wr, width(q), r0, kc}, ldp, 32);
            check_tile({q * BMAX, r0, width(q), wr, r0, kc}, ldp, 32);
        }
        for (int64_t p = 0; p < R; ++p)
            for (int64_t q = 0; q < R; ++q)
                if (p != r && q != r) check_tile({p * BMAX, q * BMAX, width(p), width(q), r0, kc}, ldp, 32);
    }
}

// The general kernel's rounds for one graph and team configuration.
static void model_general(int64_t n, int cfg, int64_t scratch_elems, int kc_wave) {
    const int BS = cfg == kGroupTiles128 ? 128 : 64;
    const int64_t ldp = (n + BS - 1) / BS * BS;
    CHECK(ldp * ldp <= scratch_elems);
    const int64_t R = ldp / BS, nt = R - 1;
    const int chunk2 = cfg == kWaveTiles64 ? kc_wave : 16;
    for (int64_t r = 0; r < R; ++r) {
        const int64_t r0 = r * BS;
        const int64_t kc = r + 1 < R ? BS : (n - r0 + 31) / 32 * 32;
        CHECK(kc >= 32 && kc <= BS && kc % 16 == 0);
        for (int64_t t = 0; t < 2 * nt; ++t) {
            int64_t q = t < nt ? t : t - nt;
            q += q >= r ? 1 : 0;
            const int64_t o = q * BS;
            if (t < nt)
                check_tile({r0, o, BS, BS, r0, kc}, ldp, chunk2);
            else
                check_tile({o, r0, BS, BS, r0, kc}, ldp, chunk2);
        }
        for (int64_t t = 0; t < nt * nt; ++t) {
            int64_t ti = t / nt, tj = t % nt;
            ti += ti >= r ? 1 : 0;
            tj += tj >= r ? 1 : 0;
            check_tile({ti * BS, tj * BS, BS, BS, r0, kc}, ldp, chunk2);
        }
    }
}

// n <= 64: one wavefront, 8 x 8 per lane over a 64 x 64 block.
static void model_wave(int64_t n) {
    for (int lane = 0; lane < 64; ++lane) {
        const int tx = lane % 8, ty = lane / 8;
        for (int m = 0; m < 8; ++m)
            for (int q = 0; q < 8; ++q) {
                const int64_t i = ty * 8 + m, j = tx * 8 + q;
                CHECK(i < 64 && j < 64);
                if (i < n && j < n) CHECK(i * n + j < n * n);
            }
    }
    CHECK((n + 15) / 16 * 16 <= 64);  // k-steps
}

// ------------------------------------------------------------------ tests
static void test_plan_args() {
    const int32_t ns[3] = {10, 20, 5};
    const int64_t ok[3] = {0, 100, 500};
    int64_t end = -1;
    CHECK(plan_args_check(ns, ok, 3, nullptr, &end) == APSP_SUCCESS && end == 525);
    CHECK(plan_args_check(nullptr, nullptr, 0, nullptr, &end) == APSP_SUCCESS);
    CHECK(plan_args_check(nullptr, ok, 2, nullptr, &end) == APSP_ERROR_INVALID_ARGUMENT);
    CHECK(plan_args_check(ns, ok, -1, nullptr, &end) == APSP_ERROR_INVALID_ARGUMENT);
    const int64_t overlap[3] = {0, 96, 500};  // graph 0 ends at 100
    CHECK(plan_args_check(ns, overlap, 3, nullptr, &end) == APSP_ERROR_INVALID_ARGUMENT);
    const int64_t misaligned[3] = {0, 102, 500};
    CHECK(plan_args_check(ns, misaligned, 3, nullptr, &end) == APSP_ERROR_INVALID_ARGUMENT);
    const int64_t negative[3] = {-4, 100, 500};
    CHECK(plan_args_check(ns, negative, 3, nullptr, &end) == APSP_ERROR_INVALID_ARGUMENT);
    const int32_t bad_n[2] = {0, 1025};
    const int64_t offs2[2] = {0, 4};
    CHECK(plan_args_check(bad_n, offs2, 1, nullptr, &end) == APSP_ERROR_INVALID_ARGUMENT);
    CHECK(plan_args_check(bad_n + 1, offs2, 1, nullptr, &end) == APSP_ERROR_INVALID_ARGUMENT);
    const int8_t cfg_bad[3] = {-2, 0, 0}, cfg_bad2[3] = {4, 0, 0}, cfg_ok[3] = {-1, 3, 2};
    CHECK(plan_args_check(ns, ok, 3, cfg_bad, &end) == APSP_ERROR_INVALID_ARGUMENT);
    CHECK(plan_args_check(ns, ok, 3, cfg_bad2, &end) == APSP_ERROR_INVALID_ARGUMENT);
    CHECK(plan_args_check(ns, ok, 3, cfg_ok, &end) == APSP_SUCCESS);
}

static void test_random_batches() {
    std::mt19937_64 rng(20241203);
    for (int trial = 0; trial < 1500; ++trial) {
        const int32_t B = (int32_t)(rng() % 300);
        std::vector<int32_t> ns((size_t)B);
        std::vector<int64_t> offs((size_t)B);
        std::vector<int8_t> forced((size_t)B);
        int64_t total = 0;
        for (int32_t b = 0; b < B; ++b) {
            const int kind = (int)(rng() % 10);
            ns[b] = kind == 0 ? 1 + (int32_t)(rng() % 64) : kind == 1 ? (int32_t)(1000 + rng() % 25)
                                                                      : 1 + (int32_t)(rng() % 700);
            offs[b] = total;
            total += ((int64_t)ns[b] * ns[b] + 3) / 4 * 4 + 4 * (int64_t)(rng() % 3);
            forced[b] = (int8_t)((int)(rng() % 5) - 1);  // -1..3
        }
        const bool pred = (rng() & 1) != 0;
        const bool use_forced = (rng() % 3) == 0;
        int64_t end = 0;
        CHECK(plan_args_check(ns.data(), offs.data(), B, use_forced ? forced.data() : nullptr, &end) ==
              APSP_SUCCESS);
        std::vector<char> bytes;
        int32_t n_team = -1;
        int64_t scratch = -1;
        bool lean = false;
        auto table = [&](int64_t n) { return pred ? (n <= 256 ? kGroupTiles64 : kWaveTiles64)
                                                  : (n <= 192 ? kGroupTiles64 : kMixed128); };
        batch_meta_with(ns.data(), offs.data(), B, pred, use_forced ? forced.data() : nullptr, table, bytes, n_team,
                        scratch, lean);
        CHECK(bytes.size() >= (size_t)B * 17);
        const int32_t *order = (const int32_t *)bytes.data();
        const int32_t *mns = order + B;
        const int64_t *moffs = (const int64_t *)(bytes.data() + (size_t)B * 8);
        const int8_t *cfg = (const int8_t *)(bytes.data() + (size_t)B * 16);
        std::vector<int> seen((size_t)B, 0);
        int32_t team = 0;
        bool expect_lean = !pred;
        for (int32_t q = 0; q < B; ++q) {
            const int32_t g = order[q];
            CHECK(g >= 0 && g < B);
            if (g < 0 || g >= B) continue;
            seen[(size_t)g]++;
            CHECK(mns[g] == ns[g] && moffs[g] == offs[g]);
            if (q > 0) {
                const int32_t p = order[q - 1];
                CHECK(ns[p] > ns[g] || (ns[p] == ns[g] && p < g));  // largest first, stable
            }
            if (ns[g] > kBatchBS) {
                ++team;
                CHECK(q < n_team);
            }
        }
        for (int32_t b = 0; b < B; ++b) {
            CHECK(seen[(size_t)b] == 1);
            const int8_t want = use_forced && forced[b] >= 0 ? forced[b] : (int8_t)table(ns[b]);
            if (ns[b] > kBatchBS && want != kMixed128 && want != kGroupTiles64) expect_lean = false;
        }
        CHECK(team == n_team && lean == expect_lean);
        for (int32_t b = 0; b < B; ++b) {
            if (ns[b] <= kBatchBS) {
                model_wave(ns[b]);
                continue;
            }
            if (lean) {
                CHECK(cfg[b] == kMixed128 || cfg[b] == kGroupTiles64);
                model_lean(ns[b], cfg[b] == kGroupTiles64 ? 64 : 128, scratch);
            } else {
                CHECK(cfg[b] >= kWaveTiles64 && cfg[b] <= kGroupTiles128);  // kMixed128 runs as 128 tiles
                for (int kcw : {16, 8}) model_general(ns[b], cfg[b], scratch, kcw);
            }
        }
    }
}

static void test_tile_shapes() {
    // lean kernel (LDS DMA, 256 threads), single-graph phases 2/3 and the
    // general kernel's group tiles
    check_dma_shape(128, 128, 16, 8, 8);
    check_dma_shape(128, 64, 16, 8, 4);
    check_dma_shape(64, 128, 16, 4, 8);
    check_dma_shape(64, 64, 16, 4, 4);
    // wavefront tiles of the general kernel, 16- and 8-element k-chunks,
    // 4-byte (VW 4) and 8-byte (VW 2) elements
    for (int kc : {16, 8}) {
        check_staged_shape(64, 64, kc, 8, 8, 4);
        check_staged_shape(64, 64, kc, 8, 8, 2);
    }
    check_staged_shape(64, 64, 16, 4, 4, 2);
    check_staged_shape(128, 128, 16, 8, 8, 2);
    check_phase1_shape(64, 8, 8, 4);
    check_phase1_shape(64, 4, 4, 4);
    check_phase1_shape(128, 8, 8, 4);
    check_phase1_shape(64, 8, 8, 2);
}

int main() {
    test_plan_args();
    test_tile_shapes();
    test_random_batches();
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
