/*
 * Seeded synthetic graph generator shared by the tests, the benchmark and
 * the oracle's callers.  It holds none of the shortest-path arithmetic: it
 * only turns (seed, graph, row, column, stream) counters into weights.
 *
 * Counter-based definition (SplitMix64 finaliser, Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014):
 *
 *   mix(z)   : z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
 *              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
 *   G        = 0x9E3779B97F4A7C15
 *   row(seed, g, i, s) = mix(mix(mix(seed + G*(s+1)) + G*(g+1)) + G*(i+1))
 *   u64(seed, g, i, j, s) = mix(row(seed, g, i, s) + G*(j+1))
 *   u01(...)  = (u64(...) >> 11) * 2^-53           in [0, 1)
 *
 * Streams: s=0 edge presence, s=1 edge weight, s=2.. per-graph parameters.
 * An edge (i != j) exists iff u01(s=0) < p; its integer weight is
 * lo + u64(s=1) mod (hi - lo + 1).  The diagonal is 0; absent edges hold
 * the caller's "no edge" value.
 */
#include <stdint.h>
#include <math.h>
#include <string.h>

#define G_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

static inline uint64_t row_key(uint64_t seed, uint64_t g, uint64_t i, uint64_t s)
{
    uint64_t h = mix64(seed + G_GOLDEN * (s + 1));
    h = mix64(h + G_GOLDEN * (g + 1));
    return mix64(h + G_GOLDEN * (i + 1));
}

static inline uint64_t cell(uint64_t rk, uint64_t j)
{
    return mix64(rk + G_GOLDEN * (j + 1));
}

static inline double to_u01(uint64_t x)
{
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

uint64_t synth_u64(uint64_t seed, uint64_t g, uint64_t i, uint64_t j, uint64_t s)
{
    return cell(row_key(seed, g, i, s), j);
}

double synth_u01(uint64_t seed, uint64_t g, uint64_t i, uint64_t j, uint64_t s)
{
    return to_u01(synth_u64(seed, g, i, j, s));
}

/* Integer-weight graph, rows [r0, r1) of an n x n matrix written into out
 * (row-major, leading dimension ld).  Edge weight = lo + u64 mod (hi-lo+1),
 * plus pot[i] - pot[j] when pot is non-NULL (a vertex potential; it keeps
 * every cycle's weight equal to the sum of its unshifted weights). */
void synth_int_rows(int32_t *out, int64_t ld, uint64_t seed, uint64_t g, int64_t n,
                    int64_t r0, int64_t r1, double p, int64_t lo, int64_t hi,
                    int32_t absent, const int32_t *pot)
{
    const uint64_t span = (uint64_t)(hi - lo + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        const uint64_t kp = row_key(seed, g, (uint64_t)i, 0);
        const uint64_t kw = row_key(seed, g, (uint64_t)i, 1);
        int32_t *row = out + (i - r0) * ld;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) { row[j] = 0; continue; }
            if (to_u01(cell(kp, (uint64_t)j)) < p) {
                int64_t w = lo + (int64_t)(cell(kw, (uint64_t)j) % span);
                if (pot) w += (int64_t)pot[i] - (int64_t)pot[j];
                row[j] = (int32_t)w;
            } else {
                row[j] = absent;
            }
        }
    }
}

/* Same presence pattern and integer weights as synth_int_rows, stored as
 * float (exact: |w| < 2^24).  Absent edges are +inf. */
void synth_intf32_rows(float *out, int64_t ld, uint64_t seed, uint64_t g, int64_t n,
                       int64_t r0, int64_t r1, double p, int64_t lo, int64_t hi)
{
    const uint64_t span = (uint64_t)(hi - lo + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        const uint64_t kp = row_key(seed, g, (uint64_t)i, 0);
        const uint64_t kw = row_key(seed, g, (uint64_t)i, 1);
        float *row = out + (i - r0) * ld;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) { row[j] = 0.0f; continue; }
            if (to_u01(cell(kp, (uint64_t)j)) < p)
                row[j] = (float)(lo + (int64_t)(cell(kw, (uint64_t)j) % span));
            else
                row[j] = INFINITY;
        }
    }
}

/* Real-valued weights: lo + u01(s=1) * (hi - lo), rounded to float. */
void synth_realf32_rows(float *out, int64_t ld, uint64_t seed, uint64_t g, int64_t n,
                        int64_t r0, int64_t r1, double p, double lo, double hi)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        const uint64_t kp = row_key(seed, g, (uint64_t)i, 0);
        const uint64_t kw = row_key(seed, g, (uint64_t)i, 1);
        float *row = out + (i - r0) * ld;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) { row[j] = 0.0f; continue; }
            if (to_u01(cell(kp, (uint64_t)j)) < p)
                row[j] = (float)(lo + to_u01(cell(kw, (uint64_t)j)) * (hi - lo));
            else
                row[j] = INFINITY;
        }
    }
}
