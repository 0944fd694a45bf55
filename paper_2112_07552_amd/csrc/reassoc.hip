// reassoc.hip -- queries Q3 and Q4 of TCUDB Section 3.3 in re-associated
// form: the group-by SUM (or COUNT) over a join whose left side forms a
// single group.
//
// Lemma Q3 writes the answer as 1^T mat(A) mat(B)^T.  Multiplying the ones
// vector in first turns the left factor into a histogram over join keys,
//   hA[k] = sum of a.val over the A records with key k      (1^T X),
// and the product with B's encoding into one pass over B's records,
//   c[h]  = sum over B records b with group h of hA[b.key] * b.val,
// so neither X nor Y is ever formed: both steps stream over the records
// (HBM-bound), O(n_A + n_B) work instead of O(K N).  Q4 (the aggregate
// without GROUP BY) is the case N = 1 with every B record in group 0.
// COUNT runs alongside with integer histograms, exact.
//
// Both scatters privatise their target array in LDS when it fits (K or N up
// to 2048 entries), so few distinct keys or groups (the paper's
// microbenchmarks use 32) do not serialise on global atomics; larger arrays
// take FP64 atomics in global memory directly.  Floating-point sums are
// order-dependent at the last bits; counts are exact.
#include "internal.h"

namespace tcu {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsBins = 2048;  // 2048 x (8 + 8) B = 32 KB of LDS

__device__ inline void report(bool bad, StatusBlock *st, int which) {
    const unsigned long long mask = __ballot(bad);
    if (mask != 0ull && (threadIdx.x & 63) == 0) {
        atomicOr(&st->flags, kFlagKeyRange);
        atomicAdd(which == 0 ? &st->skipped_a : &st->skipped_b,
                  (unsigned long long)__popcll(mask));
    }
}

// hA[key] += val, hc[key] += 1 over A's records (key in [0, K)).
template <typename T, bool PRIV>
__global__ void __launch_bounds__(kThreads)
key_hist_kernel(int64_t n, const int32_t *__restrict__ key, const T *__restrict__ val, int K,
                double *__restrict__ h, unsigned long long *__restrict__ hc, StatusBlock *st) {
    __shared__ double sh[PRIV ? kLdsBins : 1];
    __shared__ unsigned long long sc[PRIV ? kLdsBins : 1];
    if (PRIV) {
        for (int i = threadIdx.x; i < K; i += kThreads) { sh[i] = 0.0; sc[i] = 0ull; }
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const int k = key[i];
        if ((unsigned)k >= (unsigned)K) { bad = true; continue; }
        const double v = val ? (double)val[i] : 1.0;
        if (PRIV) {
            atomicAdd(sh + k, v);
            atomicAdd(sc + k, 1ull);
        } else {
            unsafeAtomicAdd(h + k, v);
            atomicAdd(hc + k, 1ull);
        }
    }
    report(bad, st, 0);
    if (PRIV) {
        __syncthreads();
        for (int i = threadIdx.x; i < K; i += kThreads) {
            if (sc[i]) {
                unsafeAtomicAdd(h + i, sh[i]);
                atomicAdd(hc + i, sc[i]);
            }
        }
    }
}

// c[group] += h[key] * val, cnt[group] += hc[key] over B's records.
template <typename T, bool PRIV>
__global__ void __launch_bounds__(kThreads)
group_sum_kernel(int64_t n, const int32_t *__restrict__ key, const int32_t *__restrict__ grp,
                 const T *__restrict__ val, int K, int N, const double *__restrict__ h,
                 const unsigned long long *__restrict__ hc, double *__restrict__ c,
                 unsigned long long *__restrict__ cnt, StatusBlock *st) {
    __shared__ double sh[PRIV ? kLdsBins : 1];
    __shared__ unsigned long long sc[PRIV ? kLdsBins : 1];
    if (PRIV) {
        for (int i = threadIdx.x; i < N; i += kThreads) { sh[i] = 0.0; sc[i] = 0ull; }
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const int k = key[i], g = grp[i];
        if ((unsigned)k >= (unsigned)K || (unsigned)g >= (unsigned)N) { bad = true; continue; }
        const unsigned long long m = hc[k];
        if (m == 0ull) continue;  // no partner in A
        const double v = h[k] * (val ? (double)val[i] : 1.0);
        if (PRIV) {
            atomicAdd(sh + g, v);
            atomicAdd(sc + g, m);
        } else {
            unsafeAtomicAdd(c + g, v);
            atomicAdd(cnt + g, m);
        }
    }
    report(bad, st, 1);
    if (PRIV) {
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += kThreads) {
            if (sc[i]) {
                unsafeAtomicAdd(c + i, sh[i]);
                atomicAdd(cnt + i, sc[i]);
            }
        }
    }
}

inline unsigned stream_grid(int64_t n) {
    const int64_t g = (n + kThreads - 1) / kThreads;
    return (unsigned)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

template <typename T>
hipError_t hist_t(const tcu_relation &R, int K, double *h, unsigned long long *hc,
                  StatusBlock *st, hipStream_t s) {
    const T *v = static_cast<const T *>(R.val);
    if (K <= kLdsBins)
        key_hist_kernel<T, true><<<stream_grid(R.n), kThreads, 0, s>>>(R.n, R.key, v, K, h, hc, st);
    else
        key_hist_kernel<T, false><<<stream_grid(R.n), kThreads, 0, s>>>(R.n, R.key, v, K, h, hc, st);
    return hipGetLastError();
}

template <typename T>
hipError_t group_t(const tcu_relation &R, int K, int N, const double *h,
                   const unsigned long long *hc, double *c, unsigned long long *cnt,
                   StatusBlock *st, hipStream_t s) {
    const T *v = static_cast<const T *>(R.val);
    if (N <= kLdsBins)
        group_sum_kernel<T, true><<<stream_grid(R.n), kThreads, 0, s>>>(R.n, R.key, R.group, v, K,
                                                                         N, h, hc, c, cnt, st);
    else
        group_sum_kernel<T, false><<<stream_grid(R.n), kThreads, 0, s>>>(R.n, R.key, R.group, v,
                                                                          K, N, h, hc, c, cnt, st);
    return hipGetLastError();
}

}  // namespace

size_t row_workspace_bytes(int K, int N) {
    return sizeof(StatusBlock) + align_up((size_t)K * 8) + align_up((size_t)K * 8) +
           align_up((size_t)N * 8);
}

hipError_t run_join_agg_row(const tcu_relation &A, const tcu_relation &B, int K, int N,
                            double *c, unsigned long long *count, void *ws, hipStream_t s) {
    char *p = static_cast<char *>(ws);
    StatusBlock *st = reinterpret_cast<StatusBlock *>(p);
    p += sizeof(StatusBlock);
    double *h = reinterpret_cast<double *>(p);
    p += align_up((size_t)K * 8);
    auto *hc = reinterpret_cast<unsigned long long *>(p);
    p += align_up((size_t)K * 8);
    auto *cnt = count ? count : reinterpret_cast<unsigned long long *>(p);
    hipError_t e = launch_clear_status(st, s);
    if (e == hipSuccess) e = launch_zero_f64(h, (size_t)K, s);
    if (e == hipSuccess) e = launch_zero_f64(reinterpret_cast<double *>(hc), (size_t)K, s);
    if (e == hipSuccess) e = launch_zero_f64(c, (size_t)N, s);
    if (e == hipSuccess) e = launch_zero_f64(reinterpret_cast<double *>(cnt), (size_t)N, s);
    if (e != hipSuccess) return e;
    if (A.n) {
        e = A.dtype == TCU_F32 ? hist_t<float>(A, K, h, hc, st, s) : hist_t<double>(A, K, h, hc, st, s);
        if (e != hipSuccess) return e;
    }
    if (B.n)
        e = B.dtype == TCU_F32 ? group_t<float>(B, K, N, h, hc, c, cnt, st, s)
                               : group_t<double>(B, K, N, h, hc, c, cnt, st, s);
    return e;
}

}  // namespace tcu
