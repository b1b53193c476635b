// Internal definitions shared by the libapsp translation units (never
// installed; the public interface is include/apsp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

#include "apsp.h"

namespace apsp {

constexpr int32_t kInf32 = APSP_INF_INT32;
// int32 results at or above this are "unreachable" once a solve is done:
// reachable distances stay within +-2^28 (weight bound), while any sum that
// involved the INF sentinel stays above INF - 2 * 2^28 > 2^29.
constexpr int32_t kFakeThreshold = 1 << 29;
// int32 sums are plain (wrapping) adds.  Under the weight bound no sum can
// overflow: every stored value lies in [-2^28, INF] and every sum in
// [-2^29, 2 INF].  Only a negative cycle drives values further down, and a
// wrapped sum needs an operand below -2^30.  Stored values never increase
// (each update is a minimum), and before any value drops below -2^29 the
// padding rows and columns hold values >= 0, so the first such value, and
// with it a witness below this bound, lands on a real (i, j) and stays
// there: a result below kWrapWitness means a negative cycle, and so does a
// negative diagonal when nothing wrapped.
constexpr int32_t kWrapWitness = -(1 << 29);
constexpr int kMaxN = 65536;

// Largest |w| accepted for int32 weights (and for exact key arithmetic on
// integer float32 weights) at size n: (n-1)|w| < 2^28.
__host__ __device__ inline int64_t weight_bound(int64_t n) {
    return n <= 1 ? (int64_t(1) << 28) - 1 : ((int64_t(1) << 28) - 1) / (n - 1);
}

void sweep_retired(bool wait);

// Single-graph solve with optional caller-provided work memory (ws may be
// null: the per-(device, stream) cache is used).  Arguments already checked.
apsp_status_t solve_internal(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype, hipStream_t s,
                             const apsp_options_t &opt, void *ws, size_t ws_bytes);
// Work memory solve_internal needs for (n, pred) with automatic block size
// and a 16-byte aligned dist.
size_t solve_work_bytes(int64_t n, apsp_dtype_t dtype, bool with_pred);
// Steppers with lent work memory and destruction without
// stream synchronisation, for the server.
apsp_status_t stepper_create(int64_t n, apsp_dtype_t dtype, bool want_pred, const apsp_options_t *options,
                             bool lend, void *ws, size_t ws_bytes, apsp_stepper_t **out);
apsp_status_t stepper_destroy(apsp_stepper_t *p, bool sync);

// Batched launch on caller-owned metadata (see apsp_batched.hip).
struct BatchLaunch {
    const void *meta;       // order[batch] int32 | ns[batch] int32 | offsets[batch] int64
    int32_t batch, n_team;
    int64_t scratch_elems;  // per workgroup
    void *scratch;          // grid * scratch_elems * (4 or 8 bytes)
    int32_t *counters;      // 8 int32 (two launches' counters), zero before the first launch
    int grid;
    bool lean;              // distances in the lean kernel (one launch)
};
apsp_status_t batched_launch(const BatchLaunch &L, apsp_dtype_t dtype, bool want_pred, void *dist,
                             int32_t *pred, int32_t *status, hipStream_t s);
// Host side of a plan: the device metadata image (order | ns | offsets |
// per-graph team configuration) with the tuning table's choices; the
// host-only planning itself is apsp_batch_host.h.
void batch_meta(const int32_t *ns, const int64_t *offsets, int32_t B, apsp_dtype_t dtype, bool pred,
                const int8_t *forced, std::vector<char> &bytes, int32_t &n_team, int64_t &scratch_elems,
                bool &lean);
int batched_blocks_per_cu(apsp_dtype_t dtype, bool lean);

// ---------------------------------------------------------------------------
// Arithmetic policies.  Each supplies the element type T, the number of
// elements per 16-byte vector (VW), the path-sum operator and the minimum,
// and strip(): the transform applied to a left operand (a D(i,k) value)
// before it is added to a right operand (a D(k,j) value).
//
// Key mode carries distance and predecessor together in one double:
//   key = d * 2^S + p,   0 <= p < 2^S (p = 2^S - 1 means "none"),
// an exact integer (|key| < 2^53), +inf when unreachable.  Then
//   strip(key_ik) + key_kj = (d_ik + d_kj) * 2^S + p_kj
// is the key of the concatenated path (its last hop is the k->j path's),
// and min over keys is the lexicographic (distance, predecessor) minimum,
// i.e. exactly the canonical predecessor rule.
// ---------------------------------------------------------------------------
// relax2(c, a0, b0, a1, b1) = min(c, a0 + b0, a1 + b1): two k-steps of one
// element.  For 32-bit types the three-input minimum is written as one
// v_min3 instruction; left to itself the compiler re-associates chains of
// these minima into 3 two/three-input minima per 4 updates instead of 2.
struct ArI32 {
    using T = int32_t;
    static constexpr int VW = 4;
    static constexpr int kP1Rows256 = 16;  // 512 threads x 16 x 8 (8 x 8 spills at 1024 threads)
    static constexpr bool kWatch = false;
    static constexpr bool kStrip = false;  // strip() is the identity
    // plain add (v_add_u32 issues at twice the rate of the clamped form on
    // gfx950); see kWrapWitness for why wrapping cannot go unnoticed
    __device__ __forceinline__ T add(T a, T b) const { return (T)((uint32_t)a + (uint32_t)b); }
    __device__ __forceinline__ T mn(T a, T b) const { return a < b ? a : b; }
    __device__ __forceinline__ T strip(T a) const { return a; }
    __device__ __forceinline__ T relax2(T c, T a0, T b0, T a1, T b1) const {
        const T s0 = add(a0, b0), s1 = add(a1, b1);
        T r;
        asm("v_min3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(c), "v"(s0), "v"(s1));
        return r;
    }
    // one step, kept as its own instruction (no fusion across steps)
    __device__ __forceinline__ T relax1(T c, T a, T b) const {
        T r = mn(c, add(a, b));
        asm("" : "+v"(r));  // materialise this step's value: no fusion across steps
        return r;
    }
};

// Floating-point minima are written as the bare instruction: fmin() with
// IEEE semantics makes the compiler quiet signalling NaNs first (one
// v_max per loop-carried operand), and no operand here is ever NaN.
__device__ __forceinline__ float vmin_f32(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double vmin_f64(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

struct ArF32 {
    using T = float;
    static constexpr int VW = 4;
    static constexpr int kP1Rows256 = 8;  // 1024 threads x 8 x 8 (16 x 8 leaves the block in scratch)
    static constexpr bool kWatch = false;
    static constexpr bool kStrip = false;
    __device__ __forceinline__ T add(T a, T b) const { return a + b; }
    __device__ __forceinline__ T mn(T a, T b) const { return vmin_f32(a, b); }
    __device__ __forceinline__ T strip(T a) const { return a; }
    __device__ __forceinline__ T relax2(T c, T a0, T b0, T a1, T b1) const {
        const T s0 = a0 + b0, s1 = a1 + b1;
        T r;
        asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(c), "v"(s0), "v"(s1));
        return r;
    }
    __device__ __forceinline__ T relax1(T c, T a, T b) const {
        T r = mn(c, add(a, b));
        asm("" : "+v"(r));  // materialise this step's value: no fusion across steps
        return r;
    }
};

// float32 arithmetic on integer-valued data: int32 weights converted to
// float32 (INF -> +inf).  While every operand of an addition is an integer
// of magnitude below 2^23, every sum is an integer below 2^24, exact in
// float32, so the results are those of int32 arithmetic bit for bit.  The
// operands of phase 3 are the outputs of phase 2, and those of phases 1 and
// 2 are the values phase 1 publishes, phase 1's outputs and phase 2's
// accumulator inputs: those kernels watch exactly these values (kWatch) and
// set *big when one reaches 2^23; the solve then redoes the graph in int32
// arithmetic.  Worth it because gfx950 issues v_add_f32 at twice the rate
// of v_add_u32 in this instruction mix.
struct ArF32W : ArF32 {
    static constexpr bool kWatch = true;
    int32_t *big;
    __device__ __forceinline__ bool is_big(float v) const {
        return v != __builtin_inff() && __builtin_fabsf(v) >= 8388608.0f;  // 2^23
    }
    __device__ __forceinline__ void raise() const { *big = 1; }
};

// Any value of a register block that would be unsafe as a later operand
// (watching policies only; false otherwise).
template <class Ar, int TM, int TN>
__device__ __forceinline__ bool any_big(const Ar &ar, const typename Ar::T (&c)[TM][TN]) {
    bool big = false;
    if constexpr (Ar::kWatch) {
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int n = 0; n < TN; ++n) big |= ar.is_big(c[m][n]);
    }
    return big;
}

struct ArKey {
    using T = double;
    static constexpr int VW = 2;
    static constexpr int kP1Rows256 = 16;  // unused: predecessor solves use BS <= 128
    static constexpr bool kWatch = false;
    static constexpr bool kStrip = true;
    int S;  // predecessor bits
    __device__ __forceinline__ T add(T a, T b) const { return a + b; }
    __device__ __forceinline__ T mn(T a, T b) const { return vmin_f64(a, b); }
    __device__ __forceinline__ T strip(T a) const {
        return __builtin_ldexp(__builtin_floor(__builtin_ldexp(a, -S)), S);
    }
    __device__ __forceinline__ T relax2(T c, T a0, T b0, T a1, T b1) const {
        return mn(mn(c, a0 + b0), a1 + b1);
    }
    __device__ __forceinline__ T relax1(T c, T a, T b) const {
        T r = mn(c, add(a, b));
        asm("" : "+v"(r));  // materialise this step's value: no fusion across steps
        return r;
    }
};

// Lexicographic mode for real-valued float32 weights with predecessors:
// (distance, predecessor) pairs stored side by side, compared
// lexicographically; the sum takes the right operand's predecessor.
struct alignas(8) DistPred {
    float d;
    int32_t p;
};
constexpr int32_t kLexNone = 0x7fffffff;

struct ArLexF32 {
    using T = DistPred;
    static constexpr int VW = 2;
    static constexpr int kP1Rows256 = 16;  // unused: predecessor solves use BS <= 128
    static constexpr bool kWatch = false;
    static constexpr bool kStrip = false;
    __device__ __forceinline__ T add(T a, T b) const { return T{a.d + b.d, b.p}; }
    __device__ __forceinline__ T mn(T c, T s) const {
        const bool take = (s.d < c.d) | ((s.d == c.d) & (s.p < c.p));
        return T{take ? s.d : c.d, take ? s.p : c.p};
    }
    __device__ __forceinline__ T strip(T a) const { return a; }
    __device__ __forceinline__ T relax2(T c, T a0, T b0, T a1, T b1) const {
        return mn(mn(c, add(a0, b0)), add(a1, b1));
    }
    __device__ __forceinline__ T relax1(T c, T a, T b) const {
        T r = mn(c, add(a, b));
        asm("" : "+v"(r.d), "+v"(r.p));
        return r;
    }
};

// 16-byte vector load/store of VW elements of any 4/8-byte element type.
template <class T>
__device__ __forceinline__ void ld16(const T *p, T *out) {
    int4 v = *reinterpret_cast<const int4 *>(p);
    __builtin_memcpy(out, &v, 16);
}
template <class T>
__device__ __forceinline__ void st16(T *p, const T *in) {
    int4 v;
    __builtin_memcpy(&v, in, 16);
    *reinterpret_cast<int4 *>(p) = v;
}

// ---------------------------------------------------------------------------
// The same workgroup tile update for 4-byte elements, with the A and B
// chunks copied from global memory straight into LDS by gfx950's
// global_load_lds_dwordx4 (each lane's 16 bytes land at LDS base + 16 *
// lane): no staging registers and no LDS store instructions, which frees
// the registers for three workgroups per CU.  The two chunk buffers are
// distinct LDS arrays and the chunk loop is unrolled by two, so the
// compiler can see that the copy into one buffer never aliases the reads of
// the other and keeps the copy in flight across the computation.
//
// A chunks are stored packed (KC elements per row); the 16-byte pieces of
// row r are XOR-swizzled by ((r * KP) >> 3) & (KP - 1) (KP = pieces per
// row) so the four rows a wavefront reads at one k fall into distinct LDS
// bank groups (8 groups of 16 bytes).
//
// CPOL is the copies' cache policy (0: the default; kCpolDevice: coherent
// at device scope, for kernels whose workgroups exchange data without a
// launch boundary or a device-scope cache flush in between).
// ---------------------------------------------------------------------------
constexpr int kCpolDevice = 16;  // sc1: device scope

template <class Ar, int MT, int NT, int KC, int TM, int TN, int CPOL = 0>
struct TileProductDMA {
    using T = typename Ar::T;
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "16-byte pieces of 4- or 8-byte elements");
    static constexpr int VW = 16 / (int)sizeof(T);
    static constexpr int TX = NT / TN;
    static constexpr int TY = MT / TM;
    static constexpr int NTH = TX * TY;
    static constexpr int NWAVES = NTH / 64;
    static constexpr int GN = TN / VW;
    static constexpr int GSTRIDE = NT / GN;
    static constexpr int KP = KC / VW;               // 16-byte pieces per A row
    static constexpr int IA = MT * KC / VW / 64;     // wave copies per A chunk
    static constexpr int IB = KC * NT / VW / 64;     // wave copies per B chunk
    static_assert(GSTRIDE == TX * VW && KP >= 2 && (KP & (KP - 1)) == 0, "tile shape");
    static_assert(IA % NWAVES == 0 && IB % NWAVES == 0, "copies split evenly over wavefronts");

    struct Smem {
        T a0[MT * KC];
        T a1[MT * KC];
        T b0[KC * NT];
        T b1[KC * NT];
    };

    __device__ __forceinline__ static int swz(int row) { return ((row * KP) >> 3) & (KP - 1); }

    __device__ __forceinline__ static void copy_chunk(T *__restrict__ la, T *__restrict__ lb,
                                                      const T *__restrict__ Abase,
                                                      const T *__restrict__ Bbase, uint32_t ld) {
        copy_a(la, Abase, ld);
        copy_b(lb, Bbase, ld);
    }

    // the A chunk alone (MT rows of KC elements, swizzled) ...
    __device__ __forceinline__ static void copy_a(T *__restrict__ la, const T *__restrict__ Abase, uint32_t ld) {
        // the wavefront index is uniform: read it into a scalar register so the
        // LDS destinations (the M0 operand of each copy) need no vector registers
        const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
#pragma unroll
        for (int j = 0; j < IA / NWAVES; ++j) {
            const int i = wave * (IA / NWAVES) + j;
            const int v = i * 64 + lane;
            const int row = v / KP, piece = v % KP;
            const T *g = Abase + ((uint32_t)row * ld + (uint32_t)((piece ^ swz(row)) * VW));
            __builtin_amdgcn_global_load_lds((const void *)g,
                                             (__attribute__((address_space(3))) void *)(la + i * 64 * VW),
                                             16, 0, CPOL);
        }
    }

    // ... and the B chunk alone (KC rows of NT elements)
    __device__ __forceinline__ static void copy_b(T *__restrict__ lb, const T *__restrict__ Bbase, uint32_t ld) {
        const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
#pragma unroll
        for (int j = 0; j < IB / NWAVES; ++j) {
            const int i = wave * (IB / NWAVES) + j;
            const int v = i * 64 + lane;
            const int row = v / (NT / VW), cv = v % (NT / VW);
            const T *g = Bbase + ((uint32_t)row * ld + (uint32_t)(cv * VW));
            __builtin_amdgcn_global_load_lds((const void *)g,
                                             (__attribute__((address_space(3))) void *)(lb + i * 64 * VW),
                                             16, 0, CPOL);
        }
    }

    // wait for this wavefront's copies (vmcnt 0), then for everyone's; in
    // key mode the A chunk (left operands) then has its predecessor bits
    // stripped in place, which the copy itself cannot do
    __device__ __forceinline__ static void copies_done(T *__restrict__ la, const Ar &ar) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) expcnt(7) lgkmcnt(15)
        __syncthreads();
        if constexpr (Ar::kStrip) {
#pragma unroll
            for (int e = threadIdx.x; e < MT * KC; e += NTH) la[e] = ar.strip(la[e]);
            __syncthreads();
        }
    }

    __device__ __forceinline__ static void compute(T (&c)[TM][TN], const T *__restrict__ As,
                                                   const T *__restrict__ Bs, int tx, int ty,
                                                   const Ar &ar) {
#pragma unroll 1
        for (int kg = 0; kg < KC; kg += VW) {
            T a[TM][VW];
#pragma unroll
            for (int m = 0; m < TM; ++m) {
                const int row = ty + TY * m;
                ld16(&As[row * KC + (((kg / VW) ^ swz(row)) * VW)], a[m]);
            }
#pragma unroll
            for (int kk = 0; kk < VW; kk += 2) {
                T b0[TN], b1[TN];
#pragma unroll
                for (int g = 0; g < GN; ++g) {
                    ld16(&Bs[(kg + kk) * NT + g * GSTRIDE + tx * VW], &b0[g * VW]);
                    ld16(&Bs[(kg + kk + 1) * NT + g * GSTRIDE + tx * VW], &b1[g * VW]);
                }
#pragma unroll
                for (int m = 0; m < TM; ++m)
#pragma unroll
                    for (int n = 0; n < TN; ++n)
                        c[m][n] = ar.relax2(c[m][n], a[m][kk], b0[n], a[m][kk + 1], b1[n]);
            }
        }
    }

    // c <- min(c, A (x) B) over kcount (a multiple of 2 KC) columns of A /
    // rows of B, double-buffered through LDS.  B advances by KC rows per
    // chunk with 64-bit offsets, so K may span a whole matrix.
    __device__ __forceinline__ static void accumulate(Smem &sm, T (&c)[TM][TN], const T *__restrict__ Abase,
                                                      const T *__restrict__ Bbase, uint32_t ld, int kcount,
                                                      int tx, int ty, const Ar &ar) {
        accumulate_in(sm.a0, sm.a1, sm.b0, sm.b1, c, Abase, Bbase, ld, kcount, tx, ty, ar);
    }

    // The same on caller-provided chunk buffers (each at least MT*KC or KC*NT
    // elements).  Four distinct LDS arrays let the compiler see that the copy
    // into one buffer never aliases the reads of the other, so the copy stays
    // in flight across the computation.
    __device__ __forceinline__ static void accumulate_in(T *__restrict__ a0, T *__restrict__ a1,
                                                         T *__restrict__ b0, T *__restrict__ b1, T (&c)[TM][TN],
                                                         const T *__restrict__ Abase, const T *__restrict__ Bbase,
                                                         uint32_t ld, int kcount, int tx, int ty, const Ar &ar) {
        const int nch = kcount / KC;
        const int64_t bstep = (int64_t)KC * ld;
        copy_chunk(a0, b0, Abase, Bbase, ld);
        copies_done(a0, ar);
        for (int ch = 0; ch < nch; ch += 2) {
            copy_chunk(a1, b1, Abase + (ch + 1) * KC, Bbase + (ch + 1) * bstep, ld);
            compute(c, a0, b0, tx, ty, ar);
            copies_done(a1, ar);
            if (ch + 2 < nch) copy_chunk(a0, b0, Abase + (ch + 2) * KC, Bbase + (ch + 2) * bstep, ld);
            compute(c, a1, b1, tx, ty, ar);
            if (ch + 2 < nch) copies_done(a0, ar);
        }
    }

    // run() on caller-provided chunk buffers (see accumulate_in).
    __device__ __forceinline__ static void run_in(T *__restrict__ a0, T *__restrict__ a1, T *__restrict__ b0,
                                                  T *__restrict__ b1, T *__restrict__ D, int64_t ld64, int64_t crow,
                                                  int64_t ccol, int64_t k0, int kcount, const Ar &ar) {
        const int tid = threadIdx.x;
        const int tx = tid % TX, ty = tid / TX;
        const uint32_t ld = (uint32_t)ld64;
        T *const Cbase = D + crow * ld64 + ccol;
        const T *const Abase = D + crow * ld64 + k0;
        const T *const Bbase = D + k0 * ld64 + ccol;
        const uint32_t coff = (uint32_t)ty * ld + (uint32_t)tx * VW;
        T c[TM][TN];
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int g = 0; g < GN; ++g)
                ld16(Cbase + (coff + (uint32_t)(TY * m) * ld + g * GSTRIDE), &c[m][g * VW]);
        accumulate_in(a0, a1, b0, b1, c, Abase, Bbase, ld, kcount, tx, ty, ar);
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int g = 0; g < GN; ++g)
                st16(Cbase + (coff + (uint32_t)(TY * m) * ld + g * GSTRIDE), &c[m][g * VW]);
    }

    // WATCH: check the tile's inputs and outputs with the policy (see ArF32W)
    template <bool WATCH = false>
    __device__ __forceinline__ static void run(Smem &sm, T *__restrict__ D, int64_t ld64, int64_t crow,
                                               int64_t ccol, int64_t k0, int kcount, const Ar &ar) {
        const int tid = threadIdx.x;
        const int tx = tid % TX, ty = tid / TX;
        const uint32_t ld = (uint32_t)ld64;
        T *const Cbase = D + crow * ld64 + ccol;
        const T *const Abase = D + crow * ld64 + k0;
        const T *const Bbase = D + k0 * ld64 + ccol;
        const uint32_t coff = (uint32_t)ty * ld + (uint32_t)tx * VW;
        T c[TM][TN];
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int g = 0; g < GN; ++g)
                ld16(Cbase + (coff + (uint32_t)(TY * m) * ld + g * GSTRIDE), &c[m][g * VW]);
        // (the inputs' check raises at once: nothing live across the products)
        if constexpr (WATCH && Ar::kWatch) {
            if (any_big(ar, c)) ar.raise();
        }
        accumulate(sm, c, Abase, Bbase, ld, kcount, tx, ty, ar);
        if constexpr (WATCH && Ar::kWatch) {
            if (any_big(ar, c)) ar.raise();
        }
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int g = 0; g < GN; ++g)
                st16(Cbase + (coff + (uint32_t)(TY * m) * ld + g * GSTRIDE), &c[m][g * VW]);
    }
};

// Barrier between the LDS writes and reads of a tile step.  Workgroup mode:
// s_barrier.  Wavefront mode (one wavefront owns the tile): a wavefront's LDS
// operations execute in issue order, so only the compiler must be kept from
// moving LDS accesses across this point.
template <bool WAVE>
__device__ __forceinline__ void tile_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <bool WAVE>
__device__ __forceinline__ int tile_tid() {
    return WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
}

// ---------------------------------------------------------------------------
// One workgroup's min-plus tile update
//     C[MT x NT] <- min(C, A[MT x K] (x) B[K x NT]),  (x) = (min, add)
// with C at (crow, ccol), A at (crow, k0), B at (k0, ccol) of the same
// row-major matrix D (leading dimension ld, every row 16-byte aligned).
//
// Thread (ty, tx) keeps a TM x TN block of C in registers: rows
// ty + TY*m (interleaved, so the A reads of one wavefront fall in distinct
// LDS banks) and columns g*(NT/GN) + tx*VW + e (16-byte groups, so a
// wavefront's B reads are contiguous).  A and B are staged through LDS in
// KC-wide k-chunks with 16-byte global loads, double buffered: chunk c+1 is
// fetched into registers while chunk c is consumed, one barrier per chunk.
// Two k-steps are fused per update so integer/float32 minima become
// three-input minima.
//
// In-place safety: the tile reads A and B only from global memory before it
// writes C, and C is written once at the end, so A or B may alias C when
// the workgroup owns every C element that its reads could see (the panel
// updates use a tile that spans the whole k-block in that direction).
// ---------------------------------------------------------------------------

template <class Ar, int MT, int NT, int KC, int TM, int TN, bool WAVE = false>
struct TileProduct {
    using T = typename Ar::T;
    static constexpr int VW = Ar::VW;
    static constexpr int TX = NT / TN;
    static constexpr int TY = MT / TM;
    static constexpr int NTH = TX * TY;
    static constexpr int GN = TN / VW;        // 16-byte column groups per thread
    static constexpr int GSTRIDE = NT / GN;   // column distance between groups
    static constexpr int LDA = KC + VW;       // padded LDS row of an A chunk
    static constexpr int NA = MT * KC / VW;   // 16-byte vectors per A chunk
    static constexpr int NB = KC * NT / VW;   // 16-byte vectors per B chunk
    static constexpr int PA = (NA + NTH - 1) / NTH;
    static constexpr int PB = (NB + NTH - 1) / NTH;
    static_assert(TN % VW == 0 && GSTRIDE == TX * VW, "column groups must tile NT");
    static_assert(!WAVE || NTH == 64, "a wavefront tile has 64 threads");
    static_assert(KC % VW == 0 && VW % 2 == 0, "k-chunk must be whole vectors");

    struct Smem {
        T a[2][MT * LDA];
        T b[2][KC * NT];
    };

    // A chunk from Abase (= &D[crow][kk]), B chunk from Bbase (= &D[kk][ccol]);
    // per-thread offsets are 32-bit so the loads use a scalar base address.
    __device__ __forceinline__ static void load_chunk(const T *__restrict__ Abase,
                                                      const T *__restrict__ Bbase, uint32_t ld,
                                                      T (&ra)[PA][VW], T (&rb)[PB][VW]) {
        const int tid = tile_tid<WAVE>();
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int v = tid + NTH * i;
            if (NA % NTH == 0 || v < NA) {
                const uint32_t row = v / (KC / VW), cv = v % (KC / VW);
                ld16(Abase + (row * ld + cv * VW), ra[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int v = tid + NTH * i;
            if (NB % NTH == 0 || v < NB) {
                const uint32_t row = v / (NT / VW), cv = v % (NT / VW);
                ld16(Bbase + (row * ld + cv * VW), rb[i]);
            }
        }
    }

    __device__ __forceinline__ static void store_chunk(Smem &sm, int buf, const Ar &ar, T (&ra)[PA][VW],
                                       T (&rb)[PB][VW]) {
        const int tid = tile_tid<WAVE>();
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int v = tid + NTH * i;
            if (NA % NTH == 0 || v < NA) {
                const int row = v / (KC / VW), cv = v % (KC / VW);
                T t[VW];
#pragma unroll
                for (int e = 0; e < VW; ++e) t[e] = ar.strip(ra[i][e]);
                st16(&sm.a[buf][row * LDA + cv * VW], t);
            }
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int v = tid + NTH * i;
            if (NB % NTH == 0 || v < NB) {
                const int row = v / (NT / VW), cv = v % (NT / VW);
                st16(&sm.b[buf][row * NT + cv * VW], rb[i]);
            }
        }
    }

    template <bool WATCH = false>
    __device__ __forceinline__ static void run(Smem &sm, T *__restrict__ D, int64_t ld64, int64_t crow,
                                               int64_t ccol, int64_t k0, int kcount, const Ar &ar) {
        const int tid = tile_tid<WAVE>();
        const int tx = tid % TX, ty = tid / TX;
        const uint32_t ld = (uint32_t)ld64;  // row offsets inside one tile fit in 32 bits
        T *const Cbase = D + crow * ld64 + ccol;
        const T *const Abase = D + crow * ld64 + k0;
        const T *const Bbase = D + k0 * ld64 + ccol;
        const uint32_t coff = (uint32_t)ty * ld + (uint32_t)tx * VW;
        T c[TM][TN];
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int g = 0; g < GN; ++g)
                ld16(Cbase + (coff + (uint32_t)(TY * m) * ld + g * GSTRIDE), &c[m][g * VW]);
        bool big = false;
        if constexpr (WATCH) big = any_big(ar, c);

        T ra[PA][VW], rb[PB][VW];
        const int nch = kcount / KC;
        load_chunk(Abase, Bbase, ld, ra, rb);
        store_chunk(sm, 0, ar, ra, rb);
        tile_sync<WAVE>();
        for (int ch = 0; ch < nch; ++ch) {
            const int buf = ch & 1;
            const bool more = ch + 1 < nch;
            if (more) load_chunk(Abase + (ch + 1) * KC, Bbase + (uint32_t)((ch + 1) * KC) * ld, ld, ra, rb);
            const T *As = sm.a[buf];
            const T *Bs = sm.b[buf];
#pragma unroll 1
            for (int kg = 0; kg < KC; kg += VW) {
                T a[TM][VW];
#pragma unroll
                for (int m = 0; m < TM; ++m) ld16(&As[(ty + TY * m) * LDA + kg], a[m]);
#pragma unroll
                for (int kk = 0; kk < VW; kk += 2) {
                    T b0[TN], b1[TN];
#pragma unroll
                    for (int g = 0; g < GN; ++g) {
                        ld16(&Bs[(kg + kk) * NT + g * GSTRIDE + tx * VW], &b0[g * VW]);
                        ld16(&Bs[(kg + kk + 1) * NT + g * GSTRIDE + tx * VW], &b1[g * VW]);
                    }
#pragma unroll
                    for (int m = 0; m < TM; ++m)
#pragma unroll
                        for (int n = 0; n < TN; ++n)
                            c[m][n] = ar.relax2(c[m][n], a[m][kk], b0[n], a[m][kk + 1], b1[n]);
                }
            }
            if (more) store_chunk(sm, buf ^ 1, ar, ra, rb);
            tile_sync<WAVE>();
        }
        if constexpr (WATCH && Ar::kWatch) {
            if (big || any_big(ar, c)) ar.raise();
        }
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int g = 0; g < GN; ++g)
                st16(Cbase + (coff + (uint32_t)(TY * m) * ld + g * GSTRIDE), &c[m][g * VW]);
    }
};

// Kernels take the work matrix as void* and a policy Ar; those launched for
// float32 solves with predecessors carry a second policy Alt and pick one of
// the two from a device word written by the set-up pass (exact fp64 keys
// when every weight is an integer within the bound, lexicographic pairs
// otherwise), so the launch sequence does not depend on the data.
struct NoAlt {
    using T = char;
    static constexpr int kP1Rows256 = 16;
    static constexpr bool kWatch = false;
};
template <class Ar, class Alt>
__device__ __forceinline__ bool use_alt(const int32_t *mode) {
    if constexpr (std::is_same_v<Alt, NoAlt>)
        return false;
    else
        return *mode != 0;
}

// ---------------------------------------------------------------- phase 1
// Closes the BS x BS diagonal block in place with BS sequential k-steps.
// One workgroup; thread (ty, tx) keeps the TM1 x TN1 block at rows
// ty*TM1.., columns tx*TN1.. in registers.  Before step k the owners of
// column k and row k publish them through LDS (double buffered by k parity,
// so one barrier per step suffices).  TT = 8: 8 x 8 blocks (16 x 8 for
// BS = 256 when the policy asks for it, see kP1Rows256); TT = 4: 4 x 4
// blocks, 16x more threads per element for latency-bound small solves.
template <int BS, int TT = 8, int ROWS256 = 16>
struct P1Shape {
    static constexpr int TM1 = (BS >= 256 && TT == 8) ? ROWS256 : TT;
    static constexpr int TN1 = TT;
    static constexpr int TX = BS / TN1, TY = BS / TM1, NTH = TX * TY;
    // the one workgroup's waves spread over the CU's 4 SIMDs: asking for
    // exactly that occupancy gives each wave the whole register budget
    static constexpr int kWavesPerSimd = NTH / 256 > 0 ? NTH / 256 : 1;
};

// Shape used by policy Ar (rows per thread at BS = 256 are a per-type choice).
template <class Ar, int BS, int TT>
using P1S = P1Shape<BS, TT, Ar::kP1Rows256>;

template <class Ar, int BS, int TT>
using P1Regs = typename Ar::T[P1S<Ar, BS, TT>::TM1][P1S<Ar, BS, TT>::TN1];

// The k-steps of a diagonal-block closure on a register-resident block:
// steps 0 <= k < ksteps (ksteps a multiple of 16, at most BS).
// Returns true if a watching policy (kWatch) saw a published value that is
// unsafe as an operand; always false otherwise.  colbuf and rowbuf each
// hold 4 rows of BS elements.
//
// 4-byte elements with blocks of at most 8 rows take the k-steps in pairs:
// the owners publish columns k, k+1 and rows k, k+1 as they stand before
// step k; every thread forms column k+1 and row k+1 as step k leaves them,
//     D'(i,k+1) = min(D(i,k+1), D(i,k) + D(k,k+1)),
//     D'(k+1,j) = min(D(k+1,j), D(k+1,k) + D(k,j)),
// for its own rows and columns, and applies both steps at once,
//     D''(i,j) = min(D(i,j), D(i,k) + D(k,j), D'(i,k+1) + D'(k+1,j)),
// one three-input minimum per element and one barrier per two steps.  The
// values are those of two single steps, bit for bit, for every policy
// (the same sums and minima).  Under a watching policy the derived
// D'(i,k+1) and D'(k+1,j) need no check of their own: each lies between
// a published value (watched) and the block's final value in that place
// (watched at the end), since values only decrease.
template <class Ar, int BS, bool WAVE, int TT = 8>
__device__ __forceinline__ bool phase1_steps(P1Regs<Ar, BS, TT> &c, int ksteps, const Ar &ar,
                                             typename Ar::T (*colbuf)[BS],
                                             typename Ar::T (*rowbuf)[BS]) {
    using T = typename Ar::T;
    bool big = false;
    constexpr int TM1 = P1S<Ar, BS, TT>::TM1, TN1 = P1S<Ar, BS, TT>::TN1, TX = P1S<Ar, BS, TT>::TX;
    constexpr int VW = Ar::VW;
    const int tid = tile_tid<WAVE>(), tx = tid % TX, ty = tid / TX;
    if constexpr (sizeof(T) == 4 && TM1 <= 8) {
        static_assert(TM1 % 2 == 0 && TN1 % 2 == 0, "a step pair has one owner");
        for (int kb = 0; kb < ksteps / 16; ++kb) {
#pragma unroll
            for (int kk = 0; kk < 16; kk += 2) {
                const int buf = (kk >> 1) & 1;
                T(*const cb)[BS] = colbuf + 2 * buf;
                T(*const rb)[BS] = rowbuf + 2 * buf;
                if (tx == kb * (16 / TN1) + kk / TN1) {
#pragma unroll
                    for (int m = 0; m < TM1; ++m) {
                        const T v0 = ar.strip(c[m][kk % TN1]), v1 = ar.strip(c[m][kk % TN1 + 1]);
                        if constexpr (Ar::kWatch) big |= ar.is_big(v0) | ar.is_big(v1);
                        cb[0][ty * TM1 + m] = v0;
                        cb[1][ty * TM1 + m] = v1;
                    }
                }
                if (ty == kb * (16 / TM1) + kk / TM1) {
#pragma unroll
                    for (int n = 0; n < TN1; ++n) {
                        if constexpr (Ar::kWatch)
                            big |= ar.is_big(c[kk % TM1][n]) | ar.is_big(c[kk % TM1 + 1][n]);
                        rb[0][tx * TN1 + n] = c[kk % TM1][n];
                        rb[1][tx * TN1 + n] = c[kk % TM1 + 1][n];
                    }
                }
                tile_sync<WAVE>();
                const int k = kb * 16 + kk;
                const T dk_k1 = ar.strip(rb[0][k + 1]);  // D(k, k+1) as a left operand
                const T dk1_k = ar.strip(rb[1][k]);      // D(k+1, k) as a left operand
                T a0[TM1], a1[TM1], b0[TN1], b1[TN1];
                if constexpr (TM1 % VW == 0) {
#pragma unroll
                    for (int g = 0; g < TM1 / VW; ++g) {
                        ld16(&cb[0][ty * TM1 + g * VW], &a0[g * VW]);
                        ld16(&cb[1][ty * TM1 + g * VW], &a1[g * VW]);
                    }
                } else {  // 2-row thread tiles
#pragma unroll
                    for (int m = 0; m < TM1; ++m) {
                        a0[m] = cb[0][ty * TM1 + m];
                        a1[m] = cb[1][ty * TM1 + m];
                    }
                }
                if constexpr (TN1 % VW == 0) {
#pragma unroll
                    for (int g = 0; g < TN1 / VW; ++g) {
                        ld16(&rb[0][tx * TN1 + g * VW], &b0[g * VW]);
                        ld16(&rb[1][tx * TN1 + g * VW], &b1[g * VW]);
                    }
                } else {
#pragma unroll
                    for (int n = 0; n < TN1; ++n) {
                        b0[n] = rb[0][tx * TN1 + n];
                        b1[n] = rb[1][tx * TN1 + n];
                    }
                }
#pragma unroll
                for (int m = 0; m < TM1; ++m) a1[m] = ar.mn(a1[m], ar.add(a0[m], dk_k1));
#pragma unroll
                for (int n = 0; n < TN1; ++n) b1[n] = ar.mn(b1[n], ar.add(dk1_k, b0[n]));
#pragma unroll
                for (int m = 0; m < TM1; ++m)
#pragma unroll
                    for (int n = 0; n < TN1; ++n) c[m][n] = ar.relax2(c[m][n], a0[m], b0[n], a1[m], b1[n]);
            }
        }
        return big;
    }
    // 16 steps per iteration keep every register index static: the owner of
    // column k holds it at n = k mod TN1, the owner of row k at m = k mod TM1.
    for (int kb = 0; kb < ksteps / 16; ++kb) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int buf = kk & 1;
            if (tx == kb * (16 / TN1) + kk / TN1) {
#pragma unroll
                for (int m = 0; m < TM1; ++m) {
                    const T v = ar.strip(c[m][kk % TN1]);
                    if constexpr (Ar::kWatch) big |= ar.is_big(v);
                    colbuf[buf][ty * TM1 + m] = v;
                }
            }
            if (ty == kb * (16 / TM1) + kk / TM1) {
#pragma unroll
                for (int n = 0; n < TN1; ++n) {
                    if constexpr (Ar::kWatch) big |= ar.is_big(c[kk % TM1][n]);
                    rowbuf[buf][tx * TN1 + n] = c[kk % TM1][n];
                }
            }
            tile_sync<WAVE>();
            T a[TM1], b[TN1];
#pragma unroll
            for (int g = 0; g < TM1 / VW; ++g) ld16(&colbuf[buf][ty * TM1 + g * VW], &a[g * VW]);
#pragma unroll
            for (int g = 0; g < TN1 / VW; ++g) ld16(&rowbuf[buf][tx * TN1 + g * VW], &b[g * VW]);
#pragma unroll
            for (int m = 0; m < TM1; ++m)
#pragma unroll
                for (int n = 0; n < TN1; ++n) {
                    // large blocks: keep each step's minima separate (fusing two
                    // steps into three-input minima costs a register per element)
                    if constexpr (TM1 > 8)
                        c[m][n] = ar.relax1(c[m][n], a[m], b[n]);
                    else
                        c[m][n] = ar.mn(c[m][n], ar.add(a[m], b[n]));
                }
        }
    }
    return big;
}

// Closes the BS x BS diagonal block at (r0, r0) of D in place, through its
// first ksteps vertices (a multiple of 16; fewer than BS only when the rest
// are isolated padding vertices, which cannot shorten any path).
template <class Ar, int BS, bool WAVE = false, int TT = 8>
__device__ __forceinline__ void phase1_body(typename Ar::T *__restrict__ D, int64_t ld, int64_t r0,
                                            const Ar &ar, typename Ar::T (*colbuf)[BS],
                                            typename Ar::T (*rowbuf)[BS], int ksteps = BS) {
    using T = typename Ar::T;
    constexpr int TM1 = P1S<Ar, BS, TT>::TM1, TN1 = P1S<Ar, BS, TT>::TN1, TX = P1S<Ar, BS, TT>::TX;
    constexpr int VW = Ar::VW;
    static_assert(!WAVE || P1S<Ar, BS, TT>::NTH == 64, "a wavefront closes 64 x 64 blocks");
    static_assert(TM1 % VW == 0 && TN1 % VW == 0, "whole 16-byte pieces per thread");
    const int tid = tile_tid<WAVE>(), tx = tid % TX, ty = tid / TX;
    T *const base = D + r0 * ld + r0;
    const uint32_t ldu = (uint32_t)ld;
    T c[TM1][TN1];
#pragma unroll
    for (int m = 0; m < TM1; ++m)
#pragma unroll
        for (int g = 0; g < TN1 / VW; ++g)
            ld16(base + ((uint32_t)(ty * TM1 + m) * ldu + tx * TN1 + g * VW), &c[m][g * VW]);
    const bool big = phase1_steps<Ar, BS, WAVE, TT>(c, ksteps, ar, colbuf, rowbuf);
    if constexpr (Ar::kWatch) {
        if (big || any_big(ar, c)) ar.raise();
    }
#pragma unroll
    for (int m = 0; m < TM1; ++m)
#pragma unroll
        for (int g = 0; g < TN1 / VW; ++g)
            st16(base + ((uint32_t)(ty * TM1 + m) * ldu + tx * TN1 + g * VW), &c[m][g * VW]);
}

}  // namespace apsp
