// Path reconstruction from the canonical predecessor matrix (the use the
// paper gives the path matrix in Section "Floyd-Warshall Algorithm": with
// it the shortest path itself can be recovered, not only its length).
//
// pred(i, j) is the vertex just before j on a shortest i -> j path, so the
// path from s to d is read backwards along row s: d, pred(s, d),
// pred(s, pred(s, d)), ... until s.  One thread per query; every walk is
// bounded by n steps and by the caller's buffer, so a matrix that was not
// produced by apsp_solve cannot make a thread loop or write out of bounds.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "apsp_internal.h"

namespace apsp {

__global__ void paths_kernel(const int32_t *__restrict__ pred, int64_t n, const int32_t *__restrict__ src,
                             const int32_t *__restrict__ dst, int32_t q, int32_t *__restrict__ paths,
                             int32_t max_len, int32_t *__restrict__ lengths) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q) return;
    const int64_t s = src[t], d = dst[t];
    if (s < 0 || s >= n || d < 0 || d >= n) {
        lengths[t] = APSP_PATH_BAD_QUERY;
        return;
    }
    int32_t *const out = paths + t * (int64_t)max_len;
    const int32_t *const row = pred + s * n;
    if (s != d && row[d] < 0) {
        lengths[t] = 0;  // unreachable
        return;
    }
    int32_t len = 0;
    int64_t v = d;
    for (int64_t step = 0;; ++step) {
        if (len >= max_len) {
            lengths[t] = APSP_PATH_TOO_LONG;
            return;
        }
        out[len++] = (int32_t)v;
        if (v == s) break;
        const int64_t u = row[v];
        if (u < 0 || u >= n || step + 1 >= n) {  // a chain longer than n - 1 hops has a cycle
            lengths[t] = APSP_PATH_BROKEN;
            return;
        }
        v = u;
    }
    for (int32_t a = 0, b = len - 1; a < b; ++a, --b) {  // written from d back to s
        const int32_t x = out[a];
        out[a] = out[b];
        out[b] = x;
    }
    lengths[t] = len;
}

// The paper's form of the path matrix (Section "Floyd-Warshall Algorithm"):
// an intermediate vertex of a shortest i -> j path, -1 when the path is the
// direct edge (or i == j, or j unreachable), so that a path is rebuilt
// recursively as path(i, m) + path(m, j).  From the canonical predecessor:
// pred(i, j) lies on a shortest i -> j path and is intermediate unless it is
// i itself.
__global__ void intermediate_kernel(const int32_t *__restrict__ pred, int64_t n, int32_t *__restrict__ out) {
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n;
        const int32_t p = pred[e];
        out[e] = (p < 0 || p == i) ? APSP_NO_PRED : p;
    }
}

}  // namespace apsp

using namespace apsp;

extern "C" apsp_status_t apsp_pred_to_intermediate(const int32_t *pred, int64_t n, int32_t *out,
                                                   hipStream_t stream) {
    if (n < 0 || n > kMaxN) return APSP_ERROR_INVALID_ARGUMENT;
    if (n == 0) return APSP_SUCCESS;
    if (!pred || !out) return APSP_ERROR_INVALID_ARGUMENT;
    const int64_t blocks = std::min<int64_t>((n * n + 255) / 256, 8192);
    hipLaunchKernelGGL(intermediate_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, pred, n, out);
    return hipGetLastError() == hipSuccess ? APSP_SUCCESS : APSP_ERROR_HIP;
}

extern "C" apsp_status_t apsp_paths(const int32_t *pred, int64_t n, const int32_t *src, const int32_t *dst,
                                    int32_t q, int32_t *paths, int32_t max_len, int32_t *lengths,
                                    hipStream_t stream) {
    if (q < 0 || n < 0 || n > kMaxN || max_len < 1) return APSP_ERROR_INVALID_ARGUMENT;
    if (q == 0) return APSP_SUCCESS;
    if (!pred || !src || !dst || !paths || !lengths || n == 0) return APSP_ERROR_INVALID_ARGUMENT;
    const int threads = 256;
    const int blocks = (int)(((int64_t)q + threads - 1) / threads);
    hipLaunchKernelGGL(paths_kernel, dim3(blocks), dim3(threads), 0, stream, pred, n, src, dst, q, paths,
                       max_len, lengths);
    return hipGetLastError() == hipSuccess ? APSP_SUCCESS : APSP_ERROR_HIP;
}
