// prims.hip -- device-wide building blocks of CST construction and of the
// label index: an exclusive prefix sum whose length may live in device memory
// (so a construction step never waits for the host to learn a size), a stable
// LSD radix sort of (key, value) pairs, and a word fill.
//
// Scan: a fixed number of workgroups B, each owning one contiguous chunk of
// the input.  Two launches: per-chunk sums, then every chunk scanned again
// from its base, which each workgroup sums from the chunk sums before it.
// Sums are 64-bit.  Inputs of at most 8192 items are scanned by one workgroup
// in one launch.  On request the scan also reports the largest input.
//
// Sort: 8-bit digits, least significant first.  Every wavefront owns one
// contiguous slice of the input; per pass it counts its digits, the
// digit-major table of those counts is scanned (so equal digits keep slice
// order, and slices keep input order), and each wavefront writes its slice
// again, 64 items at a time, ranking equal digits among its lanes with eight
// ballots.  Stable, so values with equal keys keep their input order.
#include "internal.h"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanMaxBlocks = 1024;
constexpr int kScanItems = 4;  // items per thread per tile of the downsweep
constexpr int64_t kScanSingleMax = 8192;  // up to this many items: one workgroup, one launch

__device__ inline int lane_id() { return threadIdx.x & (CSTM_WAVE - 1); }

__device__ inline int64_t wave_incl_scan64(int64_t x) {
    const int lane = lane_id();
    for (int o = 1; o < CSTM_WAVE; o <<= 1) {
        const int64_t y = __shfl_up(x, o, CSTM_WAVE);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ inline int64_t wave_sum64(int64_t x) {
    for (int o = CSTM_WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, CSTM_WAVE);
    return x;
}

// Exclusive prefix over the threads of a 256-thread workgroup; *block_total
// receives the sum.  Uses 8 int64 of LDS.
__device__ inline int64_t block_excl_scan(int64_t x, int64_t* lds, int64_t* block_total) {
    const int lane = lane_id(), w = threadIdx.x / CSTM_WAVE;
    const int64_t incl = wave_incl_scan64(x);
    if (lane == CSTM_WAVE - 1) lds[w] = incl;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int i = 0; i < kScanThreads / CSTM_WAVE; ++i) {
        const int64_t t = lds[i];
        before += i < w ? t : 0;
        all += t;
    }
    __syncthreads();
    *block_total = all;
    return before + incl - x;
}

// Chunk of block b when n items are split over nb blocks.
__device__ inline void chunk_of(int64_t n, int nb, int b, int64_t& lo, int64_t& hi) {
    const int64_t per = (n + nb - 1) / nb;
    lo = per * b;
    hi = lo + per < n ? lo + per : n;
    if (lo > n) lo = n;
}

__device__ inline int64_t wave_max64(int64_t x) {
    for (int o = CSTM_WAVE / 2; o > 0; o >>= 1) {
        const int64_t y = __shfl_xor(x, o, CSTM_WAVE);
        x = y > x ? y : x;
    }
    return x;
}

// Per-chunk sums into part[]; with max_out, the largest input also goes
// there (atomic maximum; the caller zeroes it).
template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T* __restrict__ in, const int64_t* __restrict__ n_dev,
                                                              int64_t n_host, int64_t* __restrict__ part,
                                                              int* __restrict__ max_out) {
    __shared__ int64_t lds[kScanThreads / CSTM_WAVE];
    __shared__ int64_t ldm[kScanThreads / CSTM_WAVE];
    const int64_t n = n_dev ? *n_dev : n_host;
    int64_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, lo, hi);
    int64_t s = 0, mx = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kScanThreads) {
        const int64_t x = (int64_t)in[i];
        s += x;
        mx = x > mx ? x : mx;
    }
    s = wave_sum64(s);
    mx = wave_max64(mx);
    if (lane_id() == 0) {
        lds[threadIdx.x / CSTM_WAVE] = s;
        ldm[threadIdx.x / CSTM_WAVE] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0, m = 0;
        for (int i = 0; i < kScanThreads / CSTM_WAVE; ++i) {
            t += lds[i];
            m = ldm[i] > m ? ldm[i] : m;
        }
        part[blockIdx.x] = t;
        if (max_out && m > 0) atomicMax(max_out, (int)m);
    }
}

// Every chunk scanned from its base, the sum of the chunk sums before it
// (each workgroup adds them up itself); the last workgroup writes the total
// to out[n] and *total_out.
template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const T* __restrict__ in, T* __restrict__ out,
                                                            const int64_t* __restrict__ n_dev, int64_t n_host,
                                                            const int64_t* __restrict__ part,
                                                            int64_t* __restrict__ total_out) {
    __shared__ int64_t lds[kScanThreads / CSTM_WAVE];
    const int64_t n = n_dev ? *n_dev : n_host;
    int64_t lo, hi;
    chunk_of(n, gridDim.x, blockIdx.x, lo, hi);
    int64_t before = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kScanThreads) before += part[i];
    before = wave_sum64(before);
    if (lane_id() == 0) lds[threadIdx.x / CSTM_WAVE] = before;
    __syncthreads();
    int64_t carry = 0;
    for (int i = 0; i < kScanThreads / CSTM_WAVE; ++i) carry += lds[i];
    __syncthreads();
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const int64_t total = carry + part[blockIdx.x];
        out[n] = (T)total;
        if (total_out) *total_out = total;
    }
    constexpr int64_t kTileItems = (int64_t)kScanThreads * kScanItems;
    for (int64_t t0 = lo; t0 < hi; t0 += kTileItems) {
        const int64_t mine = t0 + (int64_t)threadIdx.x * kScanItems;
        int64_t v[kScanItems];
        int64_t s = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            v[j] = mine + j < hi ? (int64_t)in[mine + j] : 0;
            s += v[j];
        }
        int64_t tile_total = 0;
        int64_t run = carry + block_excl_scan(s, lds, &tile_total);
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            if (mine + j < hi) out[mine + j] = (T)run;
            run += v[j];
        }
        carry += tile_total;
    }
}

// The whole scan in one workgroup, for short inputs: one launch instead of three.
template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_single(const T* __restrict__ in, T* __restrict__ out,
                                                              const int64_t* __restrict__ n_dev, int64_t n_host,
                                                              int64_t* __restrict__ total_out, int* __restrict__ max_out) {
    __shared__ int64_t lds[kScanThreads / CSTM_WAVE];
    const int64_t n = n_dev ? *n_dev : n_host;
    int64_t carry = 0, mx = 0;
    constexpr int64_t kTileItems = (int64_t)kScanThreads * kScanItems;
    for (int64_t t0 = 0; t0 < n; t0 += kTileItems) {
        const int64_t mine = t0 + (int64_t)threadIdx.x * kScanItems;
        int64_t v[kScanItems];
        int64_t s = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            v[j] = mine + j < n ? (int64_t)in[mine + j] : 0;
            s += v[j];
            mx = v[j] > mx ? v[j] : mx;
        }
        int64_t tile_total = 0;
        int64_t run = carry + block_excl_scan(s, lds, &tile_total);
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            if (mine + j < n) out[mine + j] = (T)run;
            run += v[j];
        }
        carry += tile_total;
    }
    if (threadIdx.x == 0) {
        out[n] = (T)carry;
        if (total_out) *total_out = carry;
    }
    if (max_out) {
        mx = wave_max64(mx);
        if (lane_id() == 0 && mx > 0) atomicMax(max_out, (int)mx);
    }
}

__global__ void k_fill_words(uint32_t* __restrict__ p, size_t n, uint32_t value) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// ------------------------------------------------------------------ radix sort

constexpr int kSortThreads = 256;
constexpr int kSortWavesPerBlock = kSortThreads / CSTM_WAVE;
constexpr int kRadix = 256;

__device__ inline void slice_of(int64_t n, int64_t waves, int64_t w, int64_t& lo, int64_t& hi) {
    const int64_t per = (n + waves - 1) / waves;
    lo = per * w;
    hi = lo + per < n ? lo + per : n;
    if (lo > n) lo = n;
}

// Digit counts of each wavefront's slice, digit-major: hist[d * waves + w].
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                            uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[kSortWavesPerBlock][kRadix];
    const int wl = threadIdx.x / CSTM_WAVE, lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kSortWavesPerBlock;
    const int64_t w = (int64_t)blockIdx.x * kSortWavesPerBlock + wl;
    for (int d = lane; d < kRadix; d += CSTM_WAVE) cnt[wl][d] = 0;
    __syncthreads();
    int64_t lo, hi;
    slice_of(n, waves, w, lo, hi);
    for (int64_t i = lo + lane; i < hi; i += CSTM_WAVE) atomicAdd(&cnt[wl][(keys[i] >> shift) & (kRadix - 1)], 1u);
    __syncthreads();
    for (int d = lane; d < kRadix; d += CSTM_WAVE) hist[(int64_t)d * waves + w] = cnt[wl][d];
}

// Stable scatter of each wavefront's slice, 64 items per step, from the
// scanned digit-major table.
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint64_t* __restrict__ keys_in,
                                                               const int32_t* __restrict__ vals_in, int64_t n, int shift,
                                                               const uint32_t* __restrict__ offs,
                                                               uint64_t* __restrict__ keys_out,
                                                               int32_t* __restrict__ vals_out) {
    __shared__ uint32_t base[kSortWavesPerBlock][kRadix];
    const int wl = threadIdx.x / CSTM_WAVE, lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kSortWavesPerBlock;
    const int64_t w = (int64_t)blockIdx.x * kSortWavesPerBlock + wl;
    for (int d = lane; d < kRadix; d += CSTM_WAVE) base[wl][d] = offs[(int64_t)d * waves + w];
    __syncthreads();
    int64_t lo, hi;
    slice_of(n, waves, w, lo, hi);
    const uint64_t below = lane ? (~0ull >> (CSTM_WAVE - lane)) : 0ull;  // lanes before this one
    for (int64_t s0 = lo; s0 < hi; s0 += CSTM_WAVE) {
        const int64_t i = s0 + lane;
        const bool in = i < hi;
        const uint64_t key = in ? keys_in[i] : 0;
        const int32_t val = in ? vals_in[i] : 0;
        const uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
        // lanes holding the same digit: intersect the ballots of its eight bits
        uint64_t same = __ballot(in);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(in && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? ones : ~ones;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        const bool leader = in && rank == 0;
        uint32_t pos = 0;
        if (in) pos = base[wl][d] + rank;
        __builtin_amdgcn_wave_barrier();
        if (leader) base[wl][d] += (uint32_t)__popcll(same);
        __builtin_amdgcn_wave_barrier();
        if (in) {
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
    }
}

template <class T>
void scan_impl(const T* in, T* out, const int64_t* n_dev, int64_t n_host, int64_t n_bound, int64_t* total_out,
               int64_t* part, hipStream_t s, int* max_out = nullptr) {
    if (n_bound <= kScanSingleMax) {
        k_scan_single<T><<<1, kScanThreads, 0, s>>>(in, out, n_dev, n_host, total_out, max_out);
        HIP_TRY(hipGetLastError());
        return;
    }
    int64_t nb = (n_bound + 4095) / 4096;
    if (nb < 1) nb = 1;
    if (nb > kScanMaxBlocks) nb = kScanMaxBlocks;
    k_scan_reduce<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n_dev, n_host, part, max_out);
    HIP_TRY(hipGetLastError());
    k_scan_down<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n_dev, n_host, part, total_out);
    HIP_TRY(hipGetLastError());
}

}  // namespace

void cstm_dscan_i64(const int64_t* in, int64_t* out, const int64_t* n_dev, int64_t n, int64_t* total_out,
                    int64_t* part, hipStream_t s, int* max_out) {
    scan_impl<int64_t>(in, out, n_dev, n_dev ? 0 : n, n, total_out, part, s, max_out);
}

void cstm_dscan_i32(const int32_t* in, int32_t* out, const int64_t* n_dev, int64_t n, int64_t* total_out,
                    int64_t* part, hipStream_t s) {
    scan_impl<int32_t>(in, out, n_dev, n_dev ? 0 : n, n, total_out, part, s);
}

void cstm_dscan_u32(const uint32_t* in, uint32_t* out, int64_t n, int64_t* part, hipStream_t s) {
    scan_impl<uint32_t>(in, out, nullptr, n, n, nullptr, part, s);
}

void cstm_fill_words(void* p, size_t bytes, uint32_t value, hipStream_t s) {
    const size_t n = bytes / 4;
    if (!n) return;
    k_fill_words<<<cstm_blocks((int64_t)n, 256, 4096), 256, 0, s>>>((uint32_t*)p, n, value);
    HIP_TRY(hipGetLastError());
}

void cstm_radix_sort_pairs(cstm_ctx* ctx, uint64_t* keys, int32_t* vals, int64_t n, int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    CSTM_REQUIRE(n < ((int64_t)1 << 31), CSTM_EINVAL, "sort length exceeds 2^31");
    int64_t blocks = (n + 16383) / 16384;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    const int64_t waves = blocks * kSortWavesPerBlock;
    const int64_t table = waves * kRadix;
    DevArena mem;
    mem.ctx = ctx;
    uint64_t* keys2 = mem.get_n<uint64_t>(n);
    int32_t* vals2 = mem.get_n<int32_t>(n);
    uint32_t* hist = mem.get_n<uint32_t>(table + 1);
    uint32_t* offs = mem.get_n<uint32_t>(table + 1);
    int64_t* part = mem.get_n<int64_t>(kScanMaxBlocks + 1);
    uint64_t* ka = keys;
    int32_t* va = vals;
    uint64_t* kb = keys2;
    int32_t* vb = vals2;
    for (int shift = 0; shift < bits; shift += 8) {
        k_sort_hist<<<(unsigned)blocks, kSortThreads, 0, s>>>(ka, n, shift, hist);
        HIP_TRY(hipGetLastError());
        cstm_dscan_u32(hist, offs, table, part, s);
        k_sort_scatter<<<(unsigned)blocks, kSortThreads, 0, s>>>(ka, va, n, shift, offs, kb, vb);
        HIP_TRY(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        HIP_TRY(hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(vals, va, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));  // the temporaries go back to the pool
}
