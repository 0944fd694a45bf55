// ooc.hip -- the FP64 product for operands larger than device memory: a
// blocked, pipelined matrix multiplication over host-resident matrices
// (TCUDB Section 4.2.3, handling large datasets; the paper extends the
// MSplitGEMM scheme to its tensor-core operator).
//
// C (m x n) = A (m x k) * B (k x n), all three row-major in host memory.
// The device holds one b x b block of C and two b x b blocks each of A and
// B (double buffers) plus a second C block, 6 b^2 doubles in all, inside a
// caller-given device buffer; b is the largest multiple of 128 that fits.
// For every block (i, j) of C, the k-blocks stream in: block l of the A row
// panel and of the B column panel are copied host -> device on one stream
// while the FP64 matrix cores multiply block l - 1 into the C block on the
// caller's stream; the finished C block goes device -> host on a third
// stream while the next C block is computed in the other C buffer.  Events
// order the three streams (a buffer is refilled only after the product that
// read it, a C buffer is reused only after its copy-out).
//
// Host-link traffic: A is read n / b times, B m / b times, C written once,
// so the product is bound by the host link unless b is large; the paper's
// figures put this copy stage first among the operator's costs.  Host
// memory should be pinned (hipHostMalloc) for the copies to overlap.
#include "internal.h"

namespace tcu {
namespace {

struct Streams {
    hipStream_t in = nullptr, out = nullptr;
    hipEvent_t loaded[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
    hipEvent_t cdone[2] = {nullptr, nullptr}, cfree[2] = {nullptr, nullptr};
    ~Streams() {
        for (int i = 0; i < 2; ++i) {
            if (loaded[i]) (void)hipEventDestroy(loaded[i]);
            if (used[i]) (void)hipEventDestroy(used[i]);
            if (cdone[i]) (void)hipEventDestroy(cdone[i]);
            if (cfree[i]) (void)hipEventDestroy(cfree[i]);
        }
        if (in) (void)hipStreamDestroy(in);
        if (out) (void)hipStreamDestroy(out);
    }
};

#define OOC_TRY(expr)                                   \
    do {                                                \
        const hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return e_;                \
    } while (0)

}  // namespace

int64_t ooc_block(size_t dev_bytes) {
    // 6 b^2 doubles: two A blocks, two B blocks, two C blocks
    int64_t b = 128;
    while ((size_t)(b + 128) * (size_t)(b + 128) * 48 <= dev_bytes) b += 128;
    return (size_t)b * (size_t)b * 48 <= dev_bytes ? b : 0;
}

hipError_t run_gemm_f64_host(int m, int n, int k, const double *A, int64_t lda, const double *B,
                             int64_t ldb, double *C, int64_t ldc, void *dev_buf,
                             size_t dev_bytes, int64_t block, hipStream_t s) {
    const int64_t b = block;
    double *dA[2], *dB[2], *dC[2];
    double *p = static_cast<double *>(dev_buf);
    for (int i = 0; i < 2; ++i) {
        dA[i] = p;
        p += b * b;
        dB[i] = p;
        p += b * b;
        dC[i] = p;
        p += b * b;
    }
    Streams st;
    OOC_TRY(hipStreamCreateWithFlags(&st.in, hipStreamNonBlocking));
    OOC_TRY(hipStreamCreateWithFlags(&st.out, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
        OOC_TRY(hipEventCreateWithFlags(&st.loaded[i], hipEventDisableTiming));
        OOC_TRY(hipEventCreateWithFlags(&st.used[i], hipEventDisableTiming));
        OOC_TRY(hipEventCreateWithFlags(&st.cdone[i], hipEventDisableTiming));
        OOC_TRY(hipEventCreateWithFlags(&st.cfree[i], hipEventDisableTiming));
    }
    // nothing the caller queued before this call may be overtaken
    hipEvent_t start;
    OOC_TRY(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    hipError_t e = hipEventRecord(start, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(st.in, start, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(st.out, start, 0);
    (void)hipEventDestroy(start);
    OOC_TRY(e);

    bool used_rec[2] = {false, false}, cfree_rec[2] = {false, false};
    int buf = 0, cb = 0;
    for (int64_t i0 = 0; i0 < m; i0 += b) {
        const int64_t bm = m - i0 < b ? m - i0 : b;
        for (int64_t j0 = 0; j0 < n; j0 += b) {
            const int64_t bn = n - j0 < b ? n - j0 : b;
            // the C buffer must have been copied out
            if (cfree_rec[cb]) OOC_TRY(hipStreamWaitEvent(s, st.cfree[cb], 0));
            for (int64_t l0 = 0; l0 < k; l0 += b) {
                const int64_t bk = k - l0 < b ? k - l0 : b;
                // refill buffer `buf` once the product that read it is done
                if (used_rec[buf]) OOC_TRY(hipStreamWaitEvent(st.in, st.used[buf], 0));
                OOC_TRY(hipMemcpy2DAsync(dA[buf], bk * 8, A + i0 * lda + l0, lda * 8, bk * 8, bm,
                                         hipMemcpyHostToDevice, st.in));
                OOC_TRY(hipMemcpy2DAsync(dB[buf], bn * 8, B + l0 * ldb + j0, ldb * 8, bn * 8, bk,
                                         hipMemcpyHostToDevice, st.in));
                OOC_TRY(hipEventRecord(st.loaded[buf], st.in));
                OOC_TRY(hipStreamWaitEvent(s, st.loaded[buf], 0));
                OOC_TRY(launch_gemm_f64(0, 0, (int)bm, (int)bn, (int)bk, dA[buf], bk, dB[buf], bn,
                                        dC[cb], bn, s, l0 > 0));
                OOC_TRY(hipEventRecord(st.used[buf], s));
                used_rec[buf] = true;
                buf ^= 1;
            }
            if (k == 0) OOC_TRY(launch_zero_f64(dC[cb], (size_t)(bm * bn), s));
            OOC_TRY(hipEventRecord(st.cdone[cb], s));
            OOC_TRY(hipStreamWaitEvent(st.out, st.cdone[cb], 0));
            OOC_TRY(hipMemcpy2DAsync(C + i0 * ldc + j0, ldc * 8, dC[cb], bn * 8, bn * 8, bm,
                                     hipMemcpyDeviceToHost, st.out));
            OOC_TRY(hipEventRecord(st.cfree[cb], st.out));
            cfree_rec[cb] = true;
            cb ^= 1;
        }
    }
    OOC_TRY(hipStreamSynchronize(st.out));
    OOC_TRY(hipStreamSynchronize(st.in));
    return hipStreamSynchronize(s);
}

}  // namespace tcu
