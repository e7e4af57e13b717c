// sort.hip -- stable LSD radix sort of the (tile | depth) keys with their
// (view * n + Gaussian) values.
//
// Only the low 32 + ceil(log2(total tiles)) key bits are sorted (8-bit digits).
// Each pass is reduce-then-scan: per-block digit histograms, a per-digit scan
// across blocks, then a scatter in which every block ranks its 4096 keys
// stably with wavefront ballots (one ballot per digit bit on wave64), sorts
// them locally in LDS and writes them out digit run by digit run, so that
// global stores are contiguous within each run.  Stability makes the order
// of equal keys the emission order (Gaussian index ascending), so the result
// is unique and comparable bit for bit.
//
// The grid is sized by the instance capacity; blocks past the device-side
// instance count exit at once, so no host synchronisation is needed.
#include "block_ops.h"
#include "gsp_internal.h"

namespace gsp {

struct SortPass {
    const unsigned long long *keys_in;
    const uint32_t *vals_in;
    unsigned long long *keys_out;
    uint32_t *vals_out;
    uint32_t *hist;        // [bins][nblk]
    uint32_t *digit_tot;   // [bins]
    const uint32_t *counters;
    int nblk;
    int shift;
};

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(SortPass a) {
    __shared__ uint32_t h[kSortBins];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const uint32_t M = a.counters[kCntMEff];
    const size_t base = (size_t)blockIdx.x * kSortItems;
    if (base < M) {
#pragma unroll 4
        for (int r = 0; r < kSortRounds; r++) {
            const size_t k = base + (size_t)r * kSortThreads + t;
            if (k < M) {
                const uint32_t d = (uint32_t)(a.keys_in[k] >> a.shift) & (kSortBins - 1);
                atomicAdd(&h[d], 1u);
            }
        }
    }
    __syncthreads();
    a.hist[(size_t)t * a.nblk + blockIdx.x] = h[t];
}

// One block per digit: exclusive scan of that digit's counts across blocks.
__global__ __launch_bounds__(kSortThreads) void k_sort_scan(SortPass a) {
    __shared__ uint32_t scratch[kSortThreads / kWave];
    const int t = threadIdx.x;
    uint32_t *row = a.hist + (size_t)blockIdx.x * a.nblk;
    const int per = (a.nblk + kSortThreads - 1) / kSortThreads;
    const int begin = min(t * per, a.nblk), end = min(begin + per, a.nblk);
    uint32_t local = 0;
    for (int k = begin; k < end; k++) local += row[k];
    uint32_t total;
    uint32_t off = block_exclusive_scan<uint32_t, kSortThreads>(local, scratch, &total);
    for (int k = begin; k < end; k++) {
        const uint32_t x = row[k];
        row[k] = off;
        off += x;
    }
    if (t == 0) a.digit_tot[blockIdx.x] = total;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortPass a) {
    constexpr int NW = kSortThreads / kWave;
    __shared__ unsigned long long skeys[kSortItems];
    __shared__ uint32_t svals[kSortItems];
    __shared__ uint32_t dstart[kSortBins];
    __shared__ uint32_t gbase[kSortBins];
    __shared__ uint32_t run[kSortBins];
    __shared__ uint32_t wcnt[NW][kSortBins];
    __shared__ uint32_t wpre[NW][kSortBins];
    __shared__ uint32_t scratch[kSortThreads / kWave];

    const uint32_t M = a.counters[kCntMEff];
    const size_t base = (size_t)blockIdx.x * kSortItems;
    if (base >= M) return;
    const int cnt = (int)min((size_t)kSortItems, (size_t)M - base);
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int w = t / kWave;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;

    unsigned long long key[kSortRounds];
    uint32_t val[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        const int k = r * kSortThreads + t;
        key[r] = k < cnt ? a.keys_in[base + k] : 0ull;
        val[r] = k < cnt ? a.vals_in[base + k] : 0u;
    }

    // local histogram -> local digit starts
    run[t] = 0;
#pragma unroll
    for (int w2 = 0; w2 < NW; w2++) wcnt[w2][t] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        if (r * kSortThreads + t < cnt)
            atomicAdd(&run[(uint32_t)(key[r] >> a.shift) & (kSortBins - 1)], 1u);
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t excl = block_exclusive_scan<uint32_t, kSortThreads>(run[t], scratch, &tot);
    const uint32_t dex = block_exclusive_scan<uint32_t, kSortThreads>(a.digit_tot[t], scratch, &tot);
    dstart[t] = excl;
    run[t] = excl;
    gbase[t] = dex + a.hist[(size_t)t * a.nblk + blockIdx.x];
    __syncthreads();

    // stable ranking, round by round, wave by wave, lane by lane
#pragma unroll 1
    for (int r = 0; r < kSortRounds; r++) {
        const bool valid = r * kSortThreads + t < cnt;
        const uint32_t d = (uint32_t)(key[r] >> a.shift) & (kSortBins - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kSortBits; b++) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        if (!valid) peers = 0;
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && (peers & lt_mask) == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        {
            uint32_t acc = run[t];
#pragma unroll
            for (int w2 = 0; w2 < NW; w2++) {
                const uint32_t c = wcnt[w2][t];
                wcnt[w2][t] = 0;
                wpre[w2][t] = acc;
                acc += c;
            }
            run[t] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wpre[w][d] + rank;
            skeys[pos] = key[r];
            svals[pos] = val[r];
        }
    }
    __syncthreads();

    for (int i = t; i < cnt; i += kSortThreads) {
        const unsigned long long k = skeys[i];
        const uint32_t d = (uint32_t)(k >> a.shift) & (kSortBins - 1);
        const size_t dst = (size_t)gbase[d] + (uint32_t)(i - dstart[d]);
        a.keys_out[dst] = k;
        a.vals_out[dst] = svals[i];
    }
}

hipError_t launch_sort(const Layout &L, char *ws, hipStream_t s, uint64_t **keys_out,
                       uint32_t **vals_out) {
    unsigned long long *k0 = region<unsigned long long>(ws, L.keys0);
    unsigned long long *k1 = region<unsigned long long>(ws, L.keys1);
    uint32_t *v0 = region<uint32_t>(ws, L.vals0);
    uint32_t *v1 = region<uint32_t>(ws, L.vals1);
    SortPass a;
    a.hist = region<uint32_t>(ws, L.hist);
    a.digit_tot = region<uint32_t>(ws, L.digit_tot);
    a.counters = region<uint32_t>(ws, L.counters);
    a.nblk = L.nblk_sort;
    for (int p = 0; p < L.sort_passes; p++) {
        a.keys_in = (p & 1) ? k1 : k0;
        a.vals_in = (p & 1) ? v1 : v0;
        a.keys_out = (p & 1) ? k0 : k1;
        a.vals_out = (p & 1) ? v0 : v1;
        a.shift = p * kSortBits;
        hipLaunchKernelGGL(k_sort_hist, dim3(L.nblk_sort), dim3(kSortThreads), 0, s, a);
        hipLaunchKernelGGL(k_sort_scan, dim3(kSortBins), dim3(kSortThreads), 0, s, a);
        hipLaunchKernelGGL(k_sort_scatter, dim3(L.nblk_sort), dim3(kSortThreads), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const bool odd = L.sort_passes & 1;
    *keys_out = reinterpret_cast<uint64_t *>(odd ? k1 : k0);
    *vals_out = odd ? v1 : v0;
    return hipSuccess;
}

}  // namespace gsp
