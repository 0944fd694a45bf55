// dict.hip -- dictionary encoding of join and group-by columns.
//
// Section 3.1 of TCUDB builds its matrices over dom(ID), the union of the
// two relations' ID domains with k distinct values v_1, ..., v_k: a value's
// matrix column is its position in that domain.  Here the domain is sorted,
// so a value's code is its rank among the distinct values of both columns:
// codes are deterministic (independent of record order and of the GPU's
// scheduling) and ORDER BY on codes is ORDER BY on values (Section 3.4).
//
// Steps (all on the caller's stream, one synchronisation to size the sort):
//  1. insert every value into an open-addressing hash set (linear probing,
//     64-bit compare-and-swap; the table has at least twice as many slots as
//     values, so every probe sequence meets a free slot);
//  2. compact the occupied slots into a list of the distinct values;
//  3. bitonic sort of that list (padded to a power of two);
//  4. write each distinct value's rank into a code array parallel to the
//     table, then look every record's value up in the table.
// INT64_MIN marks an empty slot; a column value equal to INT64_MIN is
// handled apart (it is the smallest value, so it gets code 0 when present).
// Random-access bound: about 3 probes per value on average plus the sort's
// log^2 passes over the k distinct values.
#include "internal.h"

namespace tcu {
namespace {

constexpr int kThreads = 256;
constexpr unsigned long long kEmpty = 0x8000000000000000ull;

// MurmurHash3's 64-bit finaliser (Appleby) as the slot hash.
__device__ inline unsigned long long fmix64(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

struct DictState {
    unsigned long long count;  // distinct values other than INT64_MIN
    unsigned int has_min;      // INT64_MIN occurs
    unsigned int overflow;     // a probe sequence ran out (cannot happen by sizing)
};

__global__ void dict_clear_kernel(unsigned long long *__restrict__ table, size_t slots,
                                  DictState *st) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < slots; i += stride)
        table[i] = kEmpty;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->count = 0;
        st->has_min = 0;
        st->overflow = 0;
    }
}

__global__ void dict_insert_kernel(const long long *__restrict__ vals, int64_t n,
                                   unsigned long long *__restrict__ table,
                                   unsigned long long mask, DictState *st) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const unsigned long long v = (unsigned long long)vals[i];
    if (v == kEmpty) {
        atomicOr(&st->has_min, 1u);
        return;
    }
    unsigned long long h = fmix64(v) & mask;
    for (unsigned long long probe = 0; probe <= mask; ++probe) {
        // a plain read first: a column with few distinct values finds its
        // value already present without an atomic on a contended slot
        const unsigned long long seen = __hip_atomic_load(table + h, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
        if (seen == v) return;
        if (seen == kEmpty) {
            const unsigned long long prev = atomicCAS(table + h, kEmpty, v);
            if (prev == kEmpty || prev == v) return;
        }
        h = (h + 1) & mask;
    }
    atomicOr(&st->overflow, 1u);
}

__global__ void dict_compact_kernel(const unsigned long long *__restrict__ table, size_t slots,
                                    long long *__restrict__ distinct, DictState *st) {
    const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= slots) return;
    const unsigned long long v = table[i];
    if (v != kEmpty) distinct[atomicAdd(&st->count, 1ull)] = (long long)v;
}

__global__ void dict_pad_kernel(long long *__restrict__ a, int64_t from, int64_t to) {
    const int64_t i = from + (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < to) a[i] = 0x7fffffffffffffffll;
}

// One compare-exchange pass of a bitonic sort (ascending) over a[0, P).
__global__ void bitonic_step_kernel(long long *__restrict__ a, int64_t P, int64_t j,
                                    int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= P) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const long long x = a[i], y = a[l];
    const bool ascending = (i & k) == 0;
    if ((x > y) == ascending) {
        a[i] = y;
        a[l] = x;
    }
}

__device__ inline int64_t find_slot(const unsigned long long *__restrict__ table,
                                    unsigned long long mask, unsigned long long v) {
    unsigned long long h = fmix64(v) & mask;
    for (unsigned long long probe = 0; probe <= mask; ++probe) {
        const unsigned long long t = table[h];
        if (t == v) return (int64_t)h;
        if (t == kEmpty) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

__global__ void dict_rank_kernel(const long long *__restrict__ sorted, int64_t k,
                                 const unsigned long long *__restrict__ table,
                                 unsigned long long mask, int *__restrict__ slot_code,
                                 const DictState *st, long long *__restrict__ dict) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int shift = st->has_min ? 1 : 0;
    if (r == 0 && shift) dict[0] = (long long)kEmpty;
    if (r >= k) return;
    const long long v = sorted[r];
    dict[r + shift] = v;
    const int64_t s = find_slot(table, mask, (unsigned long long)v);
    if (s >= 0) slot_code[s] = (int)(r + shift);
}

__global__ void dict_lookup_kernel(const long long *__restrict__ vals, int64_t n,
                                   const unsigned long long *__restrict__ table,
                                   unsigned long long mask, const int *__restrict__ slot_code,
                                   int *__restrict__ codes) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const unsigned long long v = (unsigned long long)vals[i];
    if (v == kEmpty) {
        codes[i] = 0;
        return;
    }
    const int64_t s = find_slot(table, mask, v);
    codes[i] = s >= 0 ? slot_code[s] : -1;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

size_t dict_table_slots(int64_t n) {
    size_t slots = 1024;
    while (slots < (size_t)(2 * n)) slots *= 2;
    return slots;
}

size_t dict_workspace_bytes(int64_t n) {
    const size_t slots = dict_table_slots(n);
    // state, table (8 B/slot), slot codes (4 B/slot), sort buffer (8 B per
    // slot / 2: the distinct values padded to a power of two <= slots / 2)
    return align_up(sizeof(DictState)) + align_up(slots * 8) + align_up(slots * 4) +
           align_up(slots / 2 * 8);
}

hipError_t run_dict_encode(const long long *a, int64_t n_a, const long long *b, int64_t n_b,
                           int *codes_a, int *codes_b, long long *dict, int64_t *k_out,
                           void *ws, hipStream_t s) {
    const int64_t n = n_a + n_b;
    const size_t slots = dict_table_slots(n);
    const unsigned long long mask = slots - 1;
    char *p = static_cast<char *>(ws);
    DictState *st = reinterpret_cast<DictState *>(p);
    p += align_up(sizeof(DictState));
    auto *table = reinterpret_cast<unsigned long long *>(p);
    p += align_up(slots * 8);
    int *slot_code = reinterpret_cast<int *>(p);
    p += align_up(slots * 4);
    long long *sorted = reinterpret_cast<long long *>(p);

    const size_t clear_blocks = (slots + kThreads - 1) / kThreads;
    const unsigned clear_grid = (unsigned)(clear_blocks < 65536 ? clear_blocks : 65536);
    dict_clear_kernel<<<clear_grid, kThreads, 0, s>>>(table, slots, st);
    if (n_a) dict_insert_kernel<<<grid_for(n_a), kThreads, 0, s>>>(a, n_a, table, mask, st);
    if (n_b) dict_insert_kernel<<<grid_for(n_b), kThreads, 0, s>>>(b, n_b, table, mask, st);
    dict_compact_kernel<<<grid_for((int64_t)slots), kThreads, 0, s>>>(table, slots, sorted, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    DictState host;
    e = hipMemcpyAsync(&host, st, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (host.overflow) return hipErrorUnknown;
    const int64_t k = (int64_t)host.count;
    int64_t P = 1;
    while (P < k) P *= 2;
    if (P > k) dict_pad_kernel<<<grid_for(P - k), kThreads, 0, s>>>(sorted, k, P);
    for (int64_t kk = 2; kk <= P; kk *= 2)
        for (int64_t j = kk / 2; j > 0; j /= 2)
            bitonic_step_kernel<<<grid_for(P), kThreads, 0, s>>>(sorted, P, j, kk);
    if (k > 0 || host.has_min)
        dict_rank_kernel<<<grid_for(k > 0 ? k : 1), kThreads, 0, s>>>(sorted, k, table, mask,
                                                                      slot_code, st, dict);
    if (n_a) dict_lookup_kernel<<<grid_for(n_a), kThreads, 0, s>>>(a, n_a, table, mask, slot_code, codes_a);
    if (n_b) dict_lookup_kernel<<<grid_for(n_b), kThreads, 0, s>>>(b, n_b, table, mask, slot_code, codes_b);
    *k_out = k + (host.has_min ? 1 : 0);
    return hipGetLastError();
}

}  // namespace tcu
