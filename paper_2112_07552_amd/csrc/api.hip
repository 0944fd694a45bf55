// api.hip -- the C ABI of libtcudb.so (declared in include/tcudb.h).
//
// Host code only: argument checks, workspace layout, and the order of the
// kernel launches that make up the operator of TCUDB Section 3.3:
//   encode A -> X, encode B -> Y (Sections 3.1/3.3), C = X * Y (Lemma Q3),
// and its adjoint.  Every launch goes to the caller's stream.
#include <string.h>

#include "internal.h"

using namespace tcu;

namespace {

tcu_status hip_status(hipError_t e) { return e == hipSuccess ? TCU_OK : TCU_ERR_HIP; }

#define TCU_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_status(e_);    \
    } while (0)

bool relation_ok(const tcu_relation *R) {
    if (R == nullptr || R->n < 0) return false;
    if (R->n > 0 && (R->group == nullptr || R->key == nullptr)) return false;
    if ((R->flags & ~TCU_REL_UNIQUE_CELLS) != 0) return false;
    return R->dtype == TCU_F64 || R->dtype == TCU_F32;
}

bool shapes_ok(int32_t M, int32_t K, int32_t N) { return M >= 1 && K >= 1 && N >= 1; }

// Workspace layout: [status block][X: M*K f64][Y: K*N f64][G: gradient]
struct Layout {
    size_t x = 0, y = 0, g = 0, total = 0;
};

Layout plan_layout(int32_t M, int32_t K, int32_t N, tcu_precision p, int flags) {
    (void)p;
    Layout L;
    size_t off = sizeof(StatusBlock);
    L.x = off;
    off += align_up((size_t)M * (size_t)K * sizeof(double));
    L.y = off;
    off += align_up((size_t)K * (size_t)N * sizeof(double));
    if (flags & TCU_WS_BACKWARD) {
        L.g = off;
        const size_t mk = (size_t)M * (size_t)K, kn = (size_t)K * (size_t)N;
        off += align_up((mk > kn ? mk : kn) * sizeof(double));
    }
    L.total = off;
    return L;
}

bool ws_ok(const void *ws, size_t ws_bytes, size_t need) {
    return ws != nullptr && ((uintptr_t)ws % kAlign) == 0 && ws_bytes >= need;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// X (M x K) and Y (K x N) from the records; `count_only` encodes ones.
hipError_t encode_both(const tcu_relation &A, const tcu_relation &B, int32_t M, int32_t K,
                       int32_t N, double *X, double *Y, StatusBlock *st, bool count_only,
                       hipStream_t s) {
    tcu_relation a = A, b = B;
    if (count_only) { a.val = nullptr; b.val = nullptr; }
    hipError_t e = launch_zero_f64(X, (size_t)M * K, s);
    if (e == hipSuccess) e = launch_zero_f64(Y, (size_t)K * N, s);
    if (e == hipSuccess) e = launch_encode(a, 0, M, K, X, st, 0, s);
    if (e == hipSuccess) e = launch_encode(b, 1, K, N, Y, st, 1, s);
    return e;
}

}  // namespace

extern "C" {

size_t tcu_workspace_bytes(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                           int32_t N, tcu_precision p, int flags) {
    (void)A; (void)B;
    if (!shapes_ok(M, K, N)) return 0;
    if (p != TCU_PREC_FP64 && p != TCU_PREC_SPLIT_BF16) return 0;
    return plan_layout(M, K, N, p, flags).total;
}

tcu_status tcu_encode(const tcu_relation *R, int transpose, int32_t rows, int32_t cols,
                      double *out, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!relation_ok(R) || rows < 1 || cols < 1 || out == nullptr) return TCU_ERR_ARG;
    if (transpose != 0 && transpose != 1) return TCU_ERR_ARG;
    if (!ws_ok(ws, ws_bytes, sizeof(StatusBlock))) return TCU_ERR_WORKSPACE;
    StatusBlock *st = at<StatusBlock>(ws, 0);
    TCU_TRY(launch_clear_status(st, stream));
    TCU_TRY(launch_zero_f64(out, (size_t)rows * (size_t)cols, stream));
    TCU_TRY(launch_encode(*R, transpose, rows, cols, out, st, 0, stream));
    return TCU_OK;
}

tcu_status tcu_gemm_f64(int trans_a, int trans_b, int32_t m, int32_t n, int32_t k,
                        const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                        int64_t ldc, hipStream_t stream) {
    if ((trans_a != 0 && trans_a != 1) || (trans_b != 0 && trans_b != 1)) return TCU_ERR_ARG;
    if (m < 0 || n < 0 || k < 0) return TCU_ERR_ARG;
    if (m == 0 || n == 0) return TCU_OK;
    if (C == nullptr || ldc < n) return TCU_ERR_ARG;
    if (k > 0) {
        if (A == nullptr || B == nullptr) return TCU_ERR_ARG;
        if (lda < (trans_a ? m : k) || ldb < (trans_b ? k : n)) return TCU_ERR_ARG;
    }
    return hip_status(launch_gemm_f64(trans_a, trans_b, m, n, k, A, lda, B, ldb, C, ldc, stream));
}

tcu_status tcu_join_agg_fwd(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, tcu_precision p, double tol, double *C, int32_t *count,
                            void *ws, size_t ws_bytes, hipStream_t stream) {
    (void)tol;
    if (!relation_ok(A) || !relation_ok(B) || !shapes_ok(M, K, N) || C == nullptr)
        return TCU_ERR_ARG;
    if (p != TCU_PREC_FP64) return TCU_ERR_ARG;
    const Layout L = plan_layout(M, K, N, p, 0);
    if (!ws_ok(ws, ws_bytes, L.total)) return TCU_ERR_WORKSPACE;
    StatusBlock *st = at<StatusBlock>(ws, 0);
    double *X = at<double>(ws, L.x), *Y = at<double>(ws, L.y);

    TCU_TRY(launch_clear_status(st, stream));
    if (count != nullptr) {
        // exact pair counts: the 0/1 (multiplicity) encodings of Section 3.1,
        // multiplied in FP64 (integers below 2^53 are exact), C as scratch
        TCU_TRY(encode_both(*A, *B, M, K, N, X, Y, nullptr, true, stream));
        TCU_TRY(launch_gemm_f64(0, 0, M, N, K, X, K, Y, N, C, N, stream));
        TCU_TRY(launch_f64_to_i32(C, count, (size_t)M * N, stream));
    }
    TCU_TRY(encode_both(*A, *B, M, K, N, X, Y, st, false, stream));
    TCU_TRY(launch_gemm_f64(0, 0, M, N, K, X, K, Y, N, C, N, stream));
    return TCU_OK;
}

tcu_status tcu_join_agg_bwd(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, tcu_precision p, double tol, const double *dC,
                            double *dA_val, double *dB_val, int flags, void *ws,
                            size_t ws_bytes, hipStream_t stream) {
    (void)tol;
    if (!relation_ok(A) || !relation_ok(B) || !shapes_ok(M, K, N) || dC == nullptr)
        return TCU_ERR_ARG;
    if ((flags & ~TCU_BWD_SAVED_ENCODINGS) != 0) return TCU_ERR_ARG;
    if (p != TCU_PREC_FP64) return TCU_ERR_ARG;
    const Layout L = plan_layout(M, K, N, p, TCU_WS_BACKWARD);
    if (!ws_ok(ws, ws_bytes, L.total)) return TCU_ERR_WORKSPACE;
    StatusBlock *st = at<StatusBlock>(ws, 0);
    double *X = at<double>(ws, L.x), *Y = at<double>(ws, L.y), *G = at<double>(ws, L.g);

    if (dA_val == nullptr && dB_val == nullptr) return TCU_OK;
    if (!(flags & TCU_BWD_SAVED_ENCODINGS)) {
        // activation checkpointing: the encodings are rebuilt from the records
        TCU_TRY(launch_clear_status(st, stream));
        TCU_TRY(encode_both(*A, *B, M, K, N, X, Y, st, false, stream));
    }
    if (dA_val != nullptr) {
        // dX = dC * Y^T (M x K), then dA.val[i] = dX[g_i, k_i]
        TCU_TRY(launch_gemm_f64(0, 1, M, K, N, dC, N, Y, N, G, K, stream));
        TCU_TRY(launch_gather(*A, 0, M, K, G, dA_val, stream));
    }
    if (dB_val != nullptr) {
        // dY = X^T * dC (K x N), then dB.val[j] = dY[k_j, h_j]
        TCU_TRY(launch_gemm_f64(1, 0, K, N, M, X, K, dC, N, G, N, stream));
        TCU_TRY(launch_gather(*B, 1, K, N, G, dB_val, stream));
    }
    return TCU_OK;
}

tcu_status tcu_sync_status(void *ws, hipStream_t stream, tcu_status_info *info) {
    if (ws == nullptr || ((uintptr_t)ws % kAlign) != 0) return TCU_ERR_WORKSPACE;
    StatusBlock host;
    TCU_TRY(hipMemcpyAsync(&host, ws, sizeof(host), hipMemcpyDeviceToHost, stream));
    TCU_TRY(hipStreamSynchronize(stream));
    if (info != nullptr) {
        info->flags = host.flags;
        info->slices = host.slices;
        info->skipped_a = host.skipped_a;
        info->skipped_b = host.skipped_b;
    }
    if (host.flags & kFlagNonFinite) return TCU_ERR_NONFINITE;
    if (host.flags & kFlagKeyRange) return TCU_ERR_KEY_RANGE;
    return TCU_OK;
}

const char *tcu_status_str(tcu_status s) {
    switch (s) {
        case TCU_OK: return "ok";
        case TCU_ERR_ARG: return "invalid argument";
        case TCU_ERR_KEY_RANGE: return "record with out-of-range key or group (skipped)";
        case TCU_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case TCU_ERR_INFEASIBLE: return "requested tolerance not reachable by the mixed form";
        case TCU_ERR_NONFINITE: return "non-finite value in the mixed form";
        case TCU_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *tcu_version(void) { return "tcudb-mi355x 0.1 (gfx950)"; }

}  // extern "C"
