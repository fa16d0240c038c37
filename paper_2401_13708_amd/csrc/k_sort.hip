// k_sort.hip -- stable LSD radix sort of (uint64 key, uint32 value) pairs for
// the tree build.
//
// Eight key bits per pass, three kernels per pass, nothing cleared with a
// memset (so the whole tree build can be captured in a HIP graph):
//  1. per tile of kTile keys, the histogram of the pass's digit (LDS
//     counters), stored digit-major: hist[d * tiles + b];
//  2. one workgroup per digit scans that digit's tile counts; every tile of
//     the scatter adds the prefix of the digit totals;
//  3. per tile, every key's stable rank among the tile's keys of its digit:
//     the tile is taken in index order (round r, wave w, lane l holds key
//     r * kBlock + 64 w + l); within a wave the lanes with the same digit are
//     found with eight ballots, and per-digit counts of the earlier waves and
//     rounds come from LDS.  Equal keys keep their input order.
#include "hts_impl.hpp"

namespace hts {

constexpr int kSortItems = 2;                   // keys per thread per tile
constexpr int kTile = kBlock * kSortItems;      // 512 keys per tile

__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                    int shift, int64_t tiles,
                                                    int32_t *__restrict__ hist) {
    __shared__ int cnt[256];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kBlock + t;
        if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & 255u)], 1);
    }
    __syncthreads();
    hist[(int64_t)t * tiles + blockIdx.x] = cnt[t];
}

// one workgroup per digit: exclusive scan of that digit's tile counts in
// place, and the digit's total
__global__ __launch_bounds__(kBlock) void k_rs_scan(int32_t *__restrict__ hist, int64_t tiles,
                                                    int32_t *__restrict__ total) {
    __shared__ int part[kBlock];
    const int t = threadIdx.x;
    int32_t *h = hist + (int64_t)blockIdx.x * tiles;
    const int64_t per = cdiv(tiles, kBlock);
    const int64_t a0 = t * per, a1 = a0 + per < tiles ? a0 + per : tiles;
    int s = 0;
    for (int64_t a = a0; a < a1; ++a) s += h[a];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const int v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t > 0 ? part[t - 1] : 0;
    for (int64_t a = a0; a < a1; ++a) {
        const int c = h[a];
        h[a] = run;
        run += c;
    }
    if (t == kBlock - 1) total[blockIdx.x] = part[kBlock - 1];
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin, int64_t n,
                                                       int shift, int64_t tiles,
                                                       const int32_t *__restrict__ offs,
                                                       const int32_t *__restrict__ total,
                                                       uint64_t *__restrict__ kout,
                                                       uint32_t *__restrict__ vout) {
    __shared__ int s_off[256];
    __shared__ int s_run[256];
    __shared__ int s_w[kBlock / kWave][256];
    const int t = threadIdx.x;
    const int w = t / kWave;
    const int lane = t & (kWave - 1);
    // start of digit t in the output: the totals of the smaller digits
    s_run[t] = total[t];
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int v = t >= o ? s_run[t - o] : 0;
        __syncthreads();
        s_run[t] += v;
        __syncthreads();
    }
    s_off[t] = (t > 0 ? s_run[t - 1] : 0) + offs[(int64_t)t * tiles + blockIdx.x];
    __syncthreads();
    s_run[t] = 0;
#pragma unroll
    for (int a = 0; a < kBlock / kWave; ++a) s_w[a][t] = 0;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kBlock + t;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0ull;
        const uint32_t val = valid ? vin[i] : 0u;
        const int dg = (int)((key >> shift) & 255u);
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(valid && ((dg >> b) & 1));
            peers &= ((dg >> b) & 1) ? ones : ~ones;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) s_w[w][dg] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = s_off[dg] + s_run[dg] + rank;
            for (int a = 0; a < w; ++a) pos += s_w[a][dg];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int a = 0; a < kBlock / kWave; ++a) {
            add += s_w[a][t];
            s_w[a][t] = 0;
        }
        s_run[t] += add;
        __syncthreads();
    }
}

size_t radix_sort_temp_bytes(int64_t n) {
    const int64_t tiles = cdiv(n, kTile);
    return (size_t)n * 8 + (size_t)n * 4 + (size_t)256 * tiles * 4 + 4096;
}

// Sorts (keys_io, vals_io) by the low `bits` key bits into (keys_out,
// vals_out); keys_io / vals_io are clobbered.  tmp holds
// radix_sort_temp_bytes(n) bytes.
hts_status radix_sort_pairs(hipStream_t st, uint64_t *keys_io, uint32_t *vals_io,
                            uint64_t *keys_out, uint32_t *vals_out, int64_t n, int bits,
                            void *tmp) {
    const int64_t tiles = cdiv(n, kTile);
    char *p = (char *)tmp;
    uint64_t *kt = (uint64_t *)p;
    uint32_t *vt = (uint32_t *)(p + (size_t)n * 8);
    int32_t *hist = (int32_t *)(p + (((size_t)n * 12 + 255) & ~(size_t)255));
    int32_t *total = hist + (size_t)256 * tiles;
    const int passes = bits < 1 ? 1 : (bits + 7) / 8;
    uint64_t *ksrc = keys_io;
    uint32_t *vsrc = vals_io;
    for (int pass = 0; pass < passes; ++pass) {
        uint64_t *kdst;
        uint32_t *vdst;
        if (pass == passes - 1) {
            kdst = keys_out;
            vdst = vals_out;
        } else if (ksrc == kt) {
            kdst = keys_io;
            vdst = vals_io;
        } else {
            kdst = kt;
            vdst = vt;
        }
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_rs_hist, dim3(tiles), dim3(kBlock), 0, st, ksrc, n, shift, tiles, hist);
        hipLaunchKernelGGL(k_rs_scan, dim3(256), dim3(kBlock), 0, st, hist, tiles, total);
        hipLaunchKernelGGL(k_rs_scatter, dim3(tiles), dim3(kBlock), 0, st, ksrc, vsrc, n, shift,
                           tiles, hist, total, kdst, vdst);
        HTS_HIP(hipGetLastError());
        ksrc = kdst;
        vsrc = vdst;
    }
    return HTS_OK;
}

}  // namespace hts
