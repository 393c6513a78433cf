// plan.hip -- device-side planning: validation and sorting of the points and
// frequencies, the staircase of the local region, the block subdivision of
// Alg. 1 (Sec. 4.1), per-block parameters and the column work items.
#include "nuht_device.h"
#include "nuht_launch.h"

#include <type_traits>

namespace nuht {

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits, of two independent segments at once (the
// points and the frequencies).  Segment s owns tiles [tile0[s], tile0[s+1])
// and elements [off[s], off[s+1]).  Launches: the keys with the first pass's
// per-tile digit counts, then per pass the counts (from the second pass on),
// their scan and the scatter.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortWaveRounds = kSortTile / kSortThreads;   // 64-key rounds per wave (= kSortRounds)

// Orders one wave's LDS accesses around it (lanes read a counter that one
// lane of the same wave then updates).
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SortSegs {
    int32_t off[3];      // element offsets of segments 0, 1 and the end
    int32_t tile0[3];    // tile offsets
    int32_t hoff[3];     // histogram offsets (256 * tiles per segment)
};

__device__ __forceinline__ int tile_segment(const SortSegs& S, int tile)
{
    return tile >= S.tile0[1] ? 1 : 0;
}

// Lanes of the wave whose digit d equals the calling lane's (8 ballots, one
// per bit), among the lanes with `valid` set.
__device__ __forceinline__ uint64_t digit_peers(int d, bool valid)
{
    uint64_t peers = __ballot(valid);
    #pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t m = __ballot((d >> b) & 1);
        peers &= ((d >> b) & 1) ? m : ~m;
    }
    return peers;
}

// Digit counts of a tile's keys held 64 per round by the waves of the block
// (digit -1: no key): in each round the lowest lane of each group of equal
// digits adds the group's size, so a digit shared by the whole round (the
// high bytes of clustered keys) costs one LDS atomic, not 64.
__device__ __forceinline__ void tile_digit_counts(const int (&dg)[kSortWaveRounds], int32_t* h)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    #pragma unroll
    for (int r = 0; r < kSortWaveRounds; ++r) {
        const bool valid = dg[r] >= 0;
        const uint64_t peers = digit_peers(dg[r], valid);
        if (valid && (peers & lt_mask) == 0) atomicAdd(&h[dg[r]], (int32_t)__popcll(peers));
    }
}

// Keys of both segments (the points, then the frequencies) in the sort's
// tiles: a nonnegative double's bit pattern, read as an unsigned integer, is
// monotone in its value, so sorting the bits sorts the values (-0.0 maps to
// 0).  Values are the caller indices within the segment.  Each tile also
// stores its digit counts for the first pass (tile-major, one row of 256 per
// tile) and errs[tile] = 1 if it holds a negative, NaN or infinite input
// (else 0).  Wave v of a tile takes its keys v * 512 .. v * 512 + 511.
__global__ __launch_bounds__(kSortThreads) void k_make_keys(const double* __restrict__ r,
                                                             const double* __restrict__ w, SortSegs S,
                                                             uint64_t* __restrict__ key, int32_t* __restrict__ val,
                                                             int32_t* __restrict__ hist, int32_t* __restrict__ errs)
{
    __shared__ int32_t h[256];
    const int tile = blockIdx.x;
    const int seg = tile_segment(S, tile);
    const int lt = tile - S.tile0[seg];
    const int base = S.off[seg], end = S.off[seg + 1];
    const double* __restrict__ x = seg ? w : r;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wbase = base + lt * kSortTile + wave * 64 * kSortWaveRounds;
    int dg[kSortWaveRounds];
    bool bad = false;
    #pragma unroll
    for (int q = 0; q < kSortWaveRounds; ++q) {
        const int i = wbase + q * 64 + lane;
        dg[q] = -1;
        if (i < end) {
            const double v = x[i - base];
            const bool ok = (v >= 0.0) && (v <= 1.7976931348623157e308);
            bad |= !ok;
            const uint64_t k = (v == 0.0 || !ok) ? 0ull : (uint64_t)__double_as_longlong(v);
            key[i] = k;
            val[i] = i - base;
            dg[q] = (int)(k & 255);
        }
    }
    h[threadIdx.x] = 0;
    __syncthreads();
    tile_digit_counts(dg, h);
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    hist[S.hoff[seg] + lt * 256 + threadIdx.x] = h[threadIdx.x];
    if (threadIdx.x == 0) errs[tile] = any_bad ? 1 : 0;
}

// Digit counts of one tile for a later pass (tile-major, one row of 256 per
// tile); wave v takes the tile's keys v * 512 .. v * 512 + 511, all loaded
// first.
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint64_t* __restrict__ key, SortSegs S,
                                                             int shift, int32_t* __restrict__ hist)
{
    __shared__ int32_t h[256];
    const int tile = blockIdx.x;
    const int seg = tile_segment(S, tile);
    const int lt = tile - S.tile0[seg];
    const int end = S.off[seg + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wbase = S.off[seg] + lt * kSortTile + wave * 64 * kSortWaveRounds;
    int dg[kSortWaveRounds];
    #pragma unroll
    for (int q = 0; q < kSortWaveRounds; ++q) {
        const int i = wbase + q * 64 + lane;
        dg[q] = i < end ? (int)((key[i] >> shift) & 255) : -1;
    }
    h[threadIdx.x] = 0;
    __syncthreads();
    tile_digit_counts(dg, h);
    __syncthreads();
    hist[S.hoff[seg] + lt * 256 + threadIdx.x] = h[threadIdx.x];
}

// 1 in *flag if any of the n tile flags is set, else 0 (one block).
__global__ __launch_bounds__(256) void k_reduce_errs(const int32_t* __restrict__ errs, int32_t n,
                                                     int32_t* __restrict__ flag)
{
    int any = 0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) any |= errs[i];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) *flag = any ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Block-wide scans (1024 threads = 16 waves): inclusive scans inside each wave
// with cross-lane shuffles, then a scan of the 16 wave totals.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = threadIdx.x & 63;
    #pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of v[q] over the block of NW waves (at most 16); tot[q]
// receives the block total.
template <class T, int NV, int NW = 16>
__device__ void block_scan(T (&v)[NV], T (&tot)[NV], T (*wsum)[16])
{
    static_assert(NW >= 1 && NW <= 16, "one wave scans the wave totals");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T incl[NV];
    #pragma unroll
    for (int q = 0; q < NV; ++q) incl[q] = wave_incl_scan(v[q]);
    if (lane == 63) {
        #pragma unroll
        for (int q = 0; q < NV; ++q) wsum[q][wave] = incl[q];
    }
    __syncthreads();
    if (wave == 0) {
        #pragma unroll
        for (int q = 0; q < NV; ++q) {
            T x = lane < NW ? wsum[q][lane] : T(0);
            x = wave_incl_scan(x);
            if (lane < NW) wsum[q][lane] = x;
        }
    }
    __syncthreads();
    #pragma unroll
    for (int q = 0; q < NV; ++q) {
        T base = wave > 0 ? wsum[q][wave - 1] : T(0);
        tot[q] = wsum[q][NW - 1];
        v[q] = base + incl[q] - v[q];
    }
    __syncthreads();
}

// Exclusive scan over the block (NW waves) of VPT consecutive values per
// thread (NV independent sequences): each thread's own running sums, then a
// block scan of the thread totals.  tot receives the block totals.
template <int NV, int VPT, int NW = 16>
__device__ void block_scan_vpt(int64_t (&v)[VPT][NV], int64_t (&tot)[NV], int64_t (*wsum)[16])
{
    int64_t t[NV];
    #pragma unroll
    for (int q = 0; q < NV; ++q) t[q] = 0;
    #pragma unroll
    for (int k = 0; k < VPT; ++k)
        #pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int64_t x = v[k][q];
            v[k][q] = t[q];
            t[q] += x;
        }
    block_scan<int64_t, NV, NW>(t, tot, wsum);
    #pragma unroll
    for (int k = 0; k < VPT; ++k)
        #pragma unroll
        for (int q = 0; q < NV; ++q) v[k][q] += t[q];
}

// Per-digit scan of the tile counts (stored tile-major: each tile's 256
// counts are one contiguous row, written and read whole by the tile's own
// histogram and scatter workgroups): one wave per (segment, digit) turns the
// digit's column of tile counts into exclusive offsets within the digit and
// stores the digit's total; the scatter adds the digits' own offsets.  The
// column is read 64 tiles at a time, all chunks' loads issued first.
constexpr int kScanChunks = 16;   // rows up to 1024 tiles in registers; longer rows loop

__global__ __launch_bounds__(256) void k_sort_scan(int32_t* __restrict__ hist, int32_t* __restrict__ dtot,
                                                   SortSegs S)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);   // seg * 256 + digit
    const int seg = row >> 8, d = row & 255;
    const int ntiles = S.tile0[seg + 1] - S.tile0[seg];
    int32_t* h = hist + S.hoff[seg] + d;     // tile i's count at h[256 i]
    int32_t run = 0;
    for (int c0 = 0; c0 < ntiles; c0 += 64 * kScanChunks) {
        int32_t v[kScanChunks];
        #pragma unroll
        for (int q = 0; q < kScanChunks; ++q) {
            const int i = c0 + q * 64 + lane;
            v[q] = i < ntiles ? h[(int64_t)i * 256] : 0;
        }
        #pragma unroll
        for (int q = 0; q < kScanChunks; ++q) {
            const int i = c0 + q * 64 + lane;
            const int32_t incl = wave_incl_scan(v[q]);
            if (i < ntiles) h[(int64_t)i * 256] = run + incl - v[q];
            run += __shfl(incl, 63);
        }
    }
    if (lane == 0) dtot[row] = run;
}

// Stable scatter through LDS.  Wave v of the block owns the tile's keys
// v * 512 .. v * 512 + 511 (in order), taken 64 at a time: each key is
// ranked among the equal digits of its 64 with wave ballots, plus the count
// of that digit in the wave's earlier keys (a wave-private counter in LDS, so
// no block barrier per round).  One block step then turns the four waves'
// digit counts into the LDS start of each (wave, digit), after the digit's
// start in the tile (an exclusive scan of the tile's counts, which are the
// differences of consecutive tile offsets in the scanned histogram).  The
// finished tile is written out with consecutive threads on consecutive
// addresses of each digit's run.
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint64_t* __restrict__ kin,
                                                                const int32_t* __restrict__ vin,
                                                                uint64_t* __restrict__ kout,
                                                                int32_t* __restrict__ vout, SortSegs S,
                                                                int shift, const int32_t* __restrict__ hist,
                                                                const int32_t* __restrict__ dtot)
{
    __shared__ uint64_t skey[kSortTile];
    __shared__ int32_t sval[kSortTile];
    __shared__ int32_t gbase[256];     // global position of the tile's first key of each digit
    __shared__ int32_t lstart[256];    // LDS start of each digit's run
    __shared__ int32_t wcnt[kSortWaves][256];   // keys of each digit per wave (running, then final)
    __shared__ int32_t tsum[2][kSortWaves];
    int tile = blockIdx.x;
    int seg = tile_segment(S, tile);
    int lt = tile - S.tile0[seg];
    int ntiles = S.tile0[seg + 1] - S.tile0[seg];
    int start = S.off[seg] + lt * kSortTile;
    int end = S.off[seg + 1];
    int lane = threadIdx.x & 63;
    int wave = threadIdx.x >> 6;
    uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // the wave's keys and values, all loaded first (one memory round trip)
    const int wbase = start + wave * 64 * kSortWaveRounds;
    uint64_t kr[kSortWaveRounds];
    int32_t vr[kSortWaveRounds];
    #pragma unroll
    for (int r = 0; r < kSortWaveRounds; ++r) {
        const int i = wbase + r * 64 + lane;
        kr[r] = i < end ? kin[i] : 0ull;
        vr[r] = i < end ? vin[i] : 0;
    }
    {
        const int d = threadIdx.x;
        const int32_t* hd = hist + S.hoff[seg] + (int64_t)lt * 256 + d;
        const int32_t tot = dtot[seg * 256 + d];
        const int32_t mine = hd[0];
        const int32_t cnt = (lt + 1 < ntiles ? hd[256] : tot) - mine;
        // exclusive scans over the digits of the segment totals and of the
        // tile counts (256 threads = 4 waves)
        int32_t it = tot, ic = cnt;
        #pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int32_t u = __shfl_up(it, o), v = __shfl_up(ic, o);
            if (lane >= o) { it += u; ic += v; }
        }
        if (lane == 63) { tsum[0][wave] = it; tsum[1][wave] = ic; }
        #pragma unroll
        for (int w2 = 0; w2 < kSortWaves; ++w2) wcnt[w2][d] = 0;
        __syncthreads();
        int32_t wt = 0, wc = 0;
        for (int w2 = 0; w2 < wave; ++w2) { wt += tsum[0][w2]; wc += tsum[1][w2]; }
        gbase[d] = S.off[seg] + wt + it - tot + mine;
        lstart[d] = wc + ic - cnt;
    }
    // ranks within the wave, in key order
    int32_t rk[kSortWaveRounds];
    int dg[kSortWaveRounds];
    int32_t* cw = wcnt[wave];
    #pragma unroll
    for (int r = 0; r < kSortWaveRounds; ++r) {
        const int i = wbase + r * 64 + lane;
        const bool valid = i < end;
        const int d = (int)((kr[r] >> shift) & 255);
        const uint64_t peers = digit_peers(d, valid);
        const int rank = __popcll(peers & lt_mask);
        const int32_t before = valid ? cw[d] : 0;
        wave_sync_lds();
        if (valid && rank == 0) cw[d] = before + __popcll(peers);
        wave_sync_lds();
        rk[r] = before + rank;
        dg[r] = valid ? d : -1;
    }
    __syncthreads();
    // LDS start of (wave, digit): the digit's start plus the earlier waves' counts
    {
        const int d = threadIdx.x;
        int32_t run = lstart[d];
        #pragma unroll
        for (int w2 = 0; w2 < kSortWaves; ++w2) {
            const int32_t c = wcnt[w2][d];
            wcnt[w2][d] = run;
            run += c;
        }
    }
    __syncthreads();
    #pragma unroll
    for (int r = 0; r < kSortWaveRounds; ++r) {
        if (dg[r] >= 0) {
            const int off = cw[dg[r]] + rk[r];
            skey[off] = kr[r];
            sval[off] = vr[r];
        }
    }
    __syncthreads();
    const int n_tile = (end - start) < kSortTile ? (end - start) : kSortTile;
    for (int q = threadIdx.x; q < n_tile; q += kSortThreads) {
        uint64_t k = skey[q];
        int d = (int)((k >> shift) & 255);
        int dst = gbase[d] + (q - lstart[d]);
        kout[dst] = k;
        vout[dst] = sval[q];
    }
}

// ---------------------------------------------------------------------------
// Sorts with fewer launches for short segments (same stable order as the LSD
// sort above, whose 25 launches dominate planning there):
// * both segments up to kSsCap keys: k_sort_small, one workgroup per segment
//   sorting it in LDS (LSD on 8-bit digits over the bits that vary);
// * both up to 2^18 keys: a splitter sort in five launches (64 bucket slots
//   per array up to 65536 keys, 1024 above) --
//   1. k_ss_sample: one workgroup per segment sorts a stratified sample of the
//      keys in LDS (bitonic for 1024 keys, LSD radix for 16384) and keeps its
//      quantiles, without repeats, as the
//      splitters u_0 < ... < u_{U-1};
//   2. k_ss_count: each tile of kSsTile keys counts its keys per bucket (range
//      bucket 2p: the keys strictly between u_{p-1} and u_p; equality bucket
//      2p + 1: the keys equal to u_p, which never need sorting) and checks its
//      inputs;
//   3. k_ss_scan: per bucket, exclusive offsets over the tiles, the bucket
//      sizes and the bucket starts;
//   4. k_ss_scatter: each tile scatters its keys, stably, into the buckets;
//   5. k_ss_local: one workgroup per bucket sorts it in LDS like k_sort_small;
//      a bucket beyond the LDS capacity (only when the sample misrepresents
//      the input) is sorted by the same workgroup through global memory.
// ---------------------------------------------------------------------------
constexpr int kSsBucketMean = 2048;      // target keys per range bucket
constexpr int kSsOversample = 32;        // sample keys per range bucket
constexpr int kSsThreads = 512;          // count and scatter workgroups: 8 waves
constexpr int kSsRounds = 16;            // 64-key rounds per wave
constexpr int kSsTile = kSsThreads * kSsRounds;
constexpr int kSsLocalThreads = 256;     // LDS sort workgroups: 4 waves
constexpr int kSsCap = kSsLocalThreads * kSsRounds;   // longest run sorted in LDS

// The splitter sort with NB bucket slots per segment (2 U + 1 <= NB - 1
// used): 64 for segments up to 65536 keys, 1024 up to 2^20.
template <int NB>
struct SsCfg {
    static constexpr int kMaxSpl = NB / 2 - 1;                          // splitters per segment at most
    static constexpr int32_t kMaxLen = (kMaxSpl + 1) * kSsBucketMean;   // longest segment
    static constexpr int kSample = kSsOversample * (kMaxSpl + 1);       // sample keys per segment at most
    static constexpr int kBits = NB == 64 ? 6 : 10;                     // bits of a bucket id
    using Id = typename std::conditional<(NB <= 256), uint8_t, uint16_t>::type;
    // scratch layout in hist (int32 units): the splitters (2 x kMaxSpl
    // uint64), their counts, the bucket starts and sizes (2 x NB each), then
    // the tile-major bucket counts
    static constexpr int kNsplOff = (4 * kMaxSpl + 63) / 64 * 64;
    static constexpr int kStartOff = kNsplOff + 64;
    static constexpr int kTotOff = kStartOff + 2 * NB;
    static constexpr int kCntOff = kTotOff + 2 * NB;
};
static_assert(SsCfg<64>::kMaxLen == 65536 && SsCfg<64>::kSample == 1024, "small splitter sort");
static_assert(SsCfg<1024>::kMaxLen == (1 << 20) && SsCfg<1024>::kSample == 16384, "large splitter sort");

// Sort key of an input (see k_make_keys); ok is false for a negative, NaN or
// infinite value, whose key is 0.
__device__ __forceinline__ uint64_t sort_key(double v, bool& ok)
{
    ok = (v >= 0.0) && (v <= 1.7976931348623157e308);
    return (v == 0.0 || !ok) ? 0ull : (uint64_t)__double_as_longlong(v);
}

// Bucket of key k among the U sorted splitters su: 2p + (k == u_p), p the
// number of splitters below k.
template <int NB>
__device__ __forceinline__ int ss_bucket(const uint64_t* su, int U, uint64_t k)
{
    int p = 0;
    #pragma unroll
    for (int step = (SsCfg<NB>::kMaxSpl + 1) / 2; step > 0; step >>= 1)
        if (p + step <= U && su[p + step - 1] < k) p += step;
    return 2 * p + ((p < U && su[p] == k) ? 1 : 0);
}

// Lanes of the wave whose bucket b (BITS bits) equals the calling lane's,
// among the lanes with `valid` set.
template <int BITS>
__device__ __forceinline__ uint64_t bucket_peers(int b, bool valid)
{
    uint64_t peers = __ballot(valid);
    #pragma unroll
    for (int i = 0; i < BITS; ++i) {
        uint64_t m = __ballot((b >> i) & 1);
        peers &= ((b >> i) & 1) ? m : ~m;
    }
    return peers;
}

// Position of sample s of ns in a segment of n keys: one point drawn from each
// of ns equal strata (a fixed hash of s picks it), so that no period of the
// input lines up with the sample.
__device__ __forceinline__ int64_t ss_sample_pos(int s, int ns, int64_t n)
{
    uint32_t h = (uint32_t)s * 0x9E3779B9u;
    h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
    const int64_t lo = ((int64_t)s * n) / ns, hi = ((int64_t)(s + 1) * n) / ns;
    return lo + (int64_t)(((uint64_t)h * (uint64_t)(hi - lo)) >> 32);
}

// Stable ranks of the 8-bit digits (key >> shift) of a workgroup's keys, held
// kSsRounds per lane in (wave, round, lane) order with `rounds` rounds per
// wave, n_valid of them: rk[q] receives the key's offset among the equal
// digits before it in its wave, wcnt[v][d] (zeroed by the caller) the count
// of digit d in wave v's keys.
__device__ __forceinline__ void ss_rank_digits(const uint64_t (&kr)[kSsRounds], int shift, int rounds, int n_valid,
                                               int32_t (*wcnt)[256], int (&dg)[kSsRounds], int (&rk)[kSsRounds])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int32_t* cw = wcnt[wave];
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        dg[q] = -1;
        if (q < rounds) {
            const int i = (wave * rounds + q) * 64 + lane;
            const bool valid = i < n_valid;
            const int d = (int)((kr[q] >> shift) & 255);
            const uint64_t peers = digit_peers(d, valid);
            const int rank = __popcll(peers & lt_mask);
            const int32_t before = valid ? cw[d] : 0;
            wave_sync_lds();
            if (valid && rank == 0) cw[d] = before + __popcll(peers);
            wave_sync_lds();
            rk[q] = before + rank;
            dg[q] = valid ? d : -1;
        }
    }
}

// Thread d of the 256: the waves' starts of digit d in wcnt (counts in,
// starts out), after the digit's start among all the keys plus base.
// Returns the digit's total.
__device__ __forceinline__ int32_t ss_digit_starts(int32_t (*wcnt)[256], int32_t base, int32_t* wtot)
{
    constexpr int kWaves = kSsLocalThreads / 64;
    const int d = threadIdx.x, lane = d & 63, wave = d >> 6;
    int32_t c = 0;
    #pragma unroll
    for (int v = 0; v < kWaves; ++v) c += wcnt[v][d];
    const int32_t incl = wave_incl_scan(c);
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    int32_t run = base + incl - c;
    for (int v = 0; v < wave; ++v) run += wtot[v];
    #pragma unroll
    for (int v = 0; v < kWaves; ++v) {
        const int32_t a = wcnt[v][d];
        wcnt[v][d] = run;
        run += a;
    }
    return c;
}

// Smallest and largest of the valid keys kr[q] over the block.
__device__ __forceinline__ void ss_key_range(const uint64_t (&kr)[kSsRounds], int rounds, int n_valid,
                                             uint64_t* red, uint64_t& kmin, uint64_t& kmax)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t lo = ~0ull, hi = 0ull;
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        const int i = (wave * rounds + q) * 64 + lane;
        if (q < rounds && i < n_valid) { lo = kr[q] < lo ? kr[q] : lo; hi = kr[q] > hi ? kr[q] : hi; }
    }
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if (lane == 0) { red[2 * wave] = lo; red[2 * wave + 1] = hi; }
    __syncthreads();
    kmin = ~0ull; kmax = 0ull;
    #pragma unroll
    for (int v = 0; v < kSsLocalThreads / 64; ++v) {
        kmin = red[2 * v] < kmin ? red[2 * v] : kmin;
        kmax = red[2 * v + 1] > kmax ? red[2 * v + 1] : kmax;
    }
    __syncthreads();
}

// LDS of a block sort of up to kSsCap keys.
struct SsBlockLds {
    uint64_t key[kSsCap];
    int32_t val[kSsCap];
    int32_t wcnt[kSsLocalThreads / 64][256];
    int32_t wtot[kSsLocalThreads / 64];
    uint64_t red[2 * (kSsLocalThreads / 64)];
};

// Rounds per wave for n keys over the block's four waves (wave-major order:
// key i sits in wave i / (64 rounds), round (i / 64) % rounds, lane i % 64).
__device__ __forceinline__ int ss_rounds(int n) { return (n + 4 * 64 - 1) / (4 * 64); }

// Stable sort of the block's n <= kSsCap keys (with their values) held in
// registers as ss_rounds(n) rounds per wave: LSD passes of 8 bits over the
// bits in which the keys differ, each ranking the keys in registers and
// exchanging them through LDS.
__device__ void ss_block_sort(uint64_t (&kr)[kSsRounds], int32_t (&vr)[kSsRounds], int n, SsBlockLds& L)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rounds = ss_rounds(n);
    int dg[kSsRounds], rk[kSsRounds];
    uint64_t kmin, kmax;
    ss_key_range(kr, rounds, n, L.red, kmin, kmax);
    const uint64_t diff = kmin ^ kmax;
    const int passes = diff ? (64 - __clzll((long long)diff) + 7) / 8 : 0;
    for (int p = 0; p < passes; ++p) {
        for (int i = threadIdx.x; i < kSsLocalThreads / 64 * 256; i += kSsLocalThreads) (&L.wcnt[0][0])[i] = 0;
        __syncthreads();
        ss_rank_digits(kr, 8 * p, rounds, n, L.wcnt, dg, rk);
        __syncthreads();
        ss_digit_starts(L.wcnt, 0, L.wtot);
        __syncthreads();
        #pragma unroll
        for (int q = 0; q < kSsRounds; ++q) {
            if (dg[q] >= 0) {
                const int off = L.wcnt[wave][dg[q]] + rk[q];
                L.key[off] = kr[q];
                L.val[off] = vr[q];
            }
        }
        __syncthreads();
        #pragma unroll
        for (int q = 0; q < kSsRounds; ++q) {
            const int i = (wave * rounds + q) * 64 + lane;
            if (q < rounds && i < n) { kr[q] = L.key[i]; vr[q] = L.val[i]; }
        }
    }
}

// Both segments at most kSsCap keys: one workgroup per segment makes the keys
// and values, sorts them in LDS into (k0, v0), and sets errs[segment] (1 if
// the segment holds a negative, NaN or infinite input).
__global__ __launch_bounds__(kSsLocalThreads) void k_sort_small(const double* __restrict__ r,
                                                                const double* __restrict__ w, SortSegs S,
                                                                uint64_t* __restrict__ k0, int32_t* __restrict__ v0,
                                                                int32_t* __restrict__ errs)
{
    __shared__ SsBlockLds L;
    const int seg = blockIdx.x;
    const int base = S.off[seg];
    const int n = S.off[seg + 1] - base;
    const double* __restrict__ x = seg ? w : r;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rounds = ss_rounds(n);
    uint64_t kr[kSsRounds];
    int32_t vr[kSsRounds];
    bool bad = false;
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        const int i = (wave * rounds + q) * 64 + lane;
        kr[q] = 0ull; vr[q] = 0;
        if (q < rounds && i < n) {
            bool ok;
            kr[q] = sort_key(x[i], ok);
            bad |= !ok;
            vr[q] = i;
        }
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (threadIdx.x == 0) errs[seg] = any_bad ? 1 : 0;
    if (n == 0) return;
    ss_block_sort(kr, vr, n, L);
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        const int i = (wave * rounds + q) * 64 + lane;
        if (q < rounds && i < n) { k0[base + i] = kr[q]; v0[base + i] = vr[q]; }
    }
}

// The B - 1 quantiles of the sorted sample sk (ns keys), each kept if it
// differs from the one before, as the segment's splitters (threads t < B - 1
// of a 1024-thread block; every thread calls it).
__device__ __forceinline__ void ss_pick_splitters(const uint64_t* sk, int ns, int B, uint64_t* spl_seg,
                                                  int32_t* nspl_seg, int32_t* wtot)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint64_t c = 0;
    bool keep = false;
    if (t < B - 1) {
        c = sk[((int64_t)(t + 1) * ns) / B];
        keep = t == 0 || c != sk[((int64_t)t * ns) / B];
    }
    const uint64_t kb = __ballot(keep);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) wtot[wave] = __popcll(kb);
    __syncthreads();
    int pos = __popcll(kb & lt_mask);
    for (int v = 0; v < wave; ++v) pos += wtot[v];
    if (keep) spl_seg[pos] = c;
    if (t == 0) {
        int tot = 0;
        for (int v = 0; v < 1024 / 64; ++v) tot += wtot[v];
        *nspl_seg = tot;
    }
}

// One workgroup of 1024 threads per segment: a stratified sample of the keys
// sorted in LDS (bitonic for the 1024-key samples of NB = 64; LSD on 8-bit
// digits over the bits that vary, 16 waves of up to 16 rounds, for the
// 16384-key samples of NB = 1024), then its quantiles as splitters.
template <int NB>
__global__ __launch_bounds__(1024) void k_ss_sample(const double* __restrict__ r, const double* __restrict__ w,
                                                    SortSegs S, uint64_t* __restrict__ spl,
                                                    int32_t* __restrict__ nspl)
{
    using C = SsCfg<NB>;
    __shared__ uint64_t sk[C::kSample];
    __shared__ int32_t wtot[16];
    const int seg = blockIdx.x;
    const int64_t n = S.off[seg + 1] - S.off[seg];
    const double* __restrict__ x = seg ? w : r;
    const int B = (int)((n + kSsBucketMean - 1) / kSsBucketMean);   // range buckets wanted
    if (B <= 1) {
        if (threadIdx.x == 0) nspl[seg] = 0;
        return;
    }
    const int ns = (int)(n < (int64_t)kSsOversample * B ? n : (int64_t)kSsOversample * B);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if constexpr (NB == 64) {
        int np2 = 1;
        while (np2 < ns) np2 <<= 1;
        {
            uint64_t k = ~0ull;
            if (t < ns) {
                bool ok;
                k = sort_key(x[ss_sample_pos(t, ns, n)], ok);
            }
            sk[t] = k;
        }
        __syncthreads();
        for (int k = 2; k <= np2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int l = t ^ j;
                if (t < np2 && l > t) {
                    const uint64_t a = sk[t], b = sk[l];
                    if ((a > b) == ((t & k) == 0)) { sk[t] = b; sk[l] = a; }
                }
                __syncthreads();
            }
    } else {
        __shared__ int32_t wcnt[16][256];
        __shared__ uint64_t red[32];
        const int rounds = (ns + 1024 - 1) / 1024;
        uint64_t kr[kSsRounds];
        #pragma unroll
        for (int q = 0; q < kSsRounds; ++q) {
            const int i = (wave * rounds + q) * 64 + lane;
            kr[q] = 0ull;
            if (q < rounds && i < ns) {
                bool ok;
                kr[q] = sort_key(x[ss_sample_pos(i, ns, n)], ok);
                sk[i] = kr[q];
            }
        }
        // the bits in which the sample's keys differ
        uint64_t lo = ~0ull, hi = 0ull;
        #pragma unroll
        for (int q = 0; q < kSsRounds; ++q) {
            const int i = (wave * rounds + q) * 64 + lane;
            if (q < rounds && i < ns) { lo = kr[q] < lo ? kr[q] : lo; hi = kr[q] > hi ? kr[q] : hi; }
        }
        #pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
            lo = a < lo ? a : lo;
            hi = b > hi ? b : hi;
        }
        if (lane == 0) { red[2 * wave] = lo; red[2 * wave + 1] = hi; }
        __syncthreads();
        uint64_t kmin = ~0ull, kmax = 0ull;
        for (int v = 0; v < 16; ++v) {
            kmin = red[2 * v] < kmin ? red[2 * v] : kmin;
            kmax = red[2 * v + 1] > kmax ? red[2 * v + 1] : kmax;
        }
        const uint64_t diff = kmin ^ kmax;
        const int passes = diff ? (64 - __clzll((long long)diff) + 7) / 8 : 0;
        int dg[kSsRounds], rk[kSsRounds];
        for (int p = 0; p < passes; ++p) {
            for (int i = t; i < 16 * 256; i += 1024) (&wcnt[0][0])[i] = 0;
            __syncthreads();
            ss_rank_digits(kr, 8 * p, rounds, ns, wcnt, dg, rk);
            __syncthreads();
            // thread d < 256: the digit's start, then the waves' starts
            int32_t c = 0, incl = 0;
            if (t < 256) {
                for (int v = 0; v < 16; ++v) c += wcnt[v][t];
                incl = wave_incl_scan(c);
                if (lane == 63) wtot[wave] = incl;
            }
            __syncthreads();
            if (t < 256) {
                int32_t run = incl - c;
                for (int v = 0; v < wave; ++v) run += wtot[v];
                for (int v = 0; v < 16; ++v) {
                    const int32_t a = wcnt[v][t];
                    wcnt[v][t] = run;
                    run += a;
                }
            }
            __syncthreads();
            #pragma unroll
            for (int q = 0; q < kSsRounds; ++q)
                if (dg[q] >= 0) sk[wcnt[wave][dg[q]] + rk[q]] = kr[q];
            __syncthreads();
            #pragma unroll
            for (int q = 0; q < kSsRounds; ++q) {
                const int i = (wave * rounds + q) * 64 + lane;
                if (q < rounds && i < ns) kr[q] = sk[i];
            }
        }
        __syncthreads();
    }
    ss_pick_splitters(sk, ns, B, spl + seg * C::kMaxSpl, nspl + seg, wtot);
}

// Per tile: the bucket counts (tile-major, NB per tile) and errs[tile] (1 if
// the tile holds a negative, NaN or infinite input).
template <int NB>
__global__ __launch_bounds__(kSsThreads) void k_ss_count(const double* __restrict__ r,
                                                         const double* __restrict__ w, SortSegs S,
                                                         const uint64_t* __restrict__ spl,
                                                         const int32_t* __restrict__ nspl,
                                                         int32_t* __restrict__ cnt, int32_t* __restrict__ errs)
{
    using C = SsCfg<NB>;
    __shared__ uint64_t su[C::kMaxSpl];
    __shared__ int32_t h[NB];
    const int tile = blockIdx.x;
    const int seg = tile_segment(S, tile);
    const int lt = tile - S.tile0[seg];
    const int base = S.off[seg], end = S.off[seg + 1];
    const int U = nspl[seg];
    const double* __restrict__ x = seg ? w : r;
    for (int i = threadIdx.x; i < U; i += kSsThreads) su[i] = spl[seg * C::kMaxSpl + i];
    for (int i = threadIdx.x; i < NB; i += kSsThreads) h[i] = 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wbase = base + lt * kSsTile + wave * 64 * kSsRounds;
    double v[kSsRounds];
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        const int i = wbase + q * 64 + lane;
        v[q] = i < end ? x[i - base] : 0.0;
    }
    __syncthreads();
    bool bad = false;
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        const int i = wbase + q * 64 + lane;
        int b = -1;
        if (i < end) {
            bool ok;
            const uint64_t k = sort_key(v[q], ok);
            bad |= !ok;
            b = ss_bucket<NB>(su, U, k);
        }
        // a bucket shared by the whole round (sorted or clustered input) costs one add
        const int b0 = __shfl(b, 0);
        const uint64_t valid = __ballot(b >= 0);
        const uint64_t same = __ballot(b >= 0 && b == b0);
        if (b0 >= 0 && same == valid) {
            if (lane == 0) atomicAdd(&h[b0], (int32_t)__popcll(valid));
        } else if (b >= 0) {
            atomicAdd(&h[b], 1);
        }
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    for (int i = threadIdx.x; i < NB; i += kSsThreads) cnt[(int64_t)tile * NB + i] = h[i];
    if (threadIdx.x == 0) errs[tile] = any_bad ? 1 : 0;
}

// Per segment, one thread per bucket: the bucket's counts over the segment's
// tiles become exclusive offsets, btot receives the bucket sizes and bstart
// their exclusive scan over the buckets (NB = 64: one wave; NB = 1024: one
// 1024-thread workgroup).
template <int NB>
__global__ __launch_bounds__(NB) void k_ss_scan(SortSegs S, int32_t* __restrict__ cnt,
                                                int32_t* __restrict__ bstart, int32_t* __restrict__ btot)
{
    const int seg = blockIdx.x, b = threadIdx.x;
    const int t0 = S.tile0[seg], nt = S.tile0[seg + 1] - t0;
    int32_t run = 0;
    for (int t = 0; t < nt; t += 16) {
        int32_t v[16];
        #pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = t + q < nt ? cnt[(int64_t)(t0 + t + q) * NB + b] : 0;
        #pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (t + q < nt) cnt[(int64_t)(t0 + t + q) * NB + b] = run;
            run += v[q];
        }
    }
    btot[seg * NB + b] = run;
    if constexpr (NB == 64) {
        bstart[seg * NB + b] = wave_incl_scan(run) - run;
    } else {
        __shared__ int32_t wsum[1][16];
        int32_t e[1] = {run}, tot[1];
        block_scan<int32_t, 1, NB / 64>(e, tot, wsum);
        bstart[seg * NB + b] = e[0];
    }
}

// Stable scatter of a tile into the buckets, through LDS: wave v owns the
// tile's keys v * 1024 .. v * 1024 + 1023 (in order), ranked 64 at a time
// among the equal buckets of their round plus the wave's earlier keys of that
// bucket; one block step turns the waves' counts into LDS starts; the staged
// tile is written out with consecutive threads on consecutive addresses of
// each bucket's run.
template <int NB>
__global__ __launch_bounds__(kSsThreads) void k_ss_scatter(const double* __restrict__ r,
                                                           const double* __restrict__ w, SortSegs S,
                                                           const uint64_t* __restrict__ spl,
                                                           const int32_t* __restrict__ nspl,
                                                           const int32_t* __restrict__ cnt,
                                                           const int32_t* __restrict__ bstart,
                                                           uint64_t* __restrict__ kout, int32_t* __restrict__ vout)
{
    using C = SsCfg<NB>;
    using Id = typename C::Id;
    constexpr int kWaves = kSsThreads / 64;
    __shared__ uint64_t skey[kSsTile];
    __shared__ int32_t sval[kSsTile];
    __shared__ Id sbk[kSsTile];
    __shared__ uint64_t su[C::kMaxSpl];
    __shared__ int32_t wcnt[kWaves][NB];
    __shared__ int32_t gbase[NB];
    __shared__ int32_t lstart[NB];
    __shared__ int32_t wtot[kWaves];
    const int tile = blockIdx.x;
    const int seg = tile_segment(S, tile);
    const int lt = tile - S.tile0[seg];
    const int base = S.off[seg], end = S.off[seg + 1];
    const int start = base + lt * kSsTile;
    const int U = nspl[seg];
    const double* __restrict__ x = seg ? w : r;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int wbase = start + wave * 64 * kSsRounds;
    uint64_t kr[kSsRounds];
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        const int i = wbase + q * 64 + lane;
        bool ok;
        kr[q] = i < end ? sort_key(x[i - base], ok) : 0ull;
    }
    for (int i = threadIdx.x; i < U; i += kSsThreads) su[i] = spl[seg * C::kMaxSpl + i];
    for (int i = threadIdx.x; i < kWaves * NB; i += kSsThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    int bk[kSsRounds], rk[kSsRounds];
    int32_t* cw = wcnt[wave];
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        const int i = wbase + q * 64 + lane;
        const bool valid = i < end;
        const int b = valid ? ss_bucket<NB>(su, U, kr[q]) : 0;
        const uint64_t peers = bucket_peers<C::kBits>(b, valid);
        const int rank = __popcll(peers & lt_mask);
        const int32_t before = valid ? cw[b] : 0;
        wave_sync_lds();
        if (valid && rank == 0) cw[b] = before + __popcll(peers);
        wave_sync_lds();
        rk[q] = before + rank;
        bk[q] = valid ? b : -1;
    }
    __syncthreads();
    // per bucket: the tile's count, its LDS start (exclusive scan over the
    // buckets), the waves' starts and the global base
    if constexpr (NB == 64) {
        if (wave == 0) {
            const int b = lane;
            int32_t c = 0;
            #pragma unroll
            for (int v = 0; v < kWaves; ++v) c += wcnt[v][b];
            const int32_t ls = wave_incl_scan(c) - c;
            lstart[b] = ls;
            int32_t run = ls;
            #pragma unroll
            for (int v = 0; v < kWaves; ++v) {
                const int32_t a = wcnt[v][b];
                wcnt[v][b] = run;
                run += a;
            }
            gbase[b] = base + bstart[seg * NB + b] + cnt[(int64_t)tile * NB + b];
        }
    } else {
        // thread t: buckets BPT t .. BPT t + BPT - 1
        constexpr int BPT = NB / kSsThreads;
        const int b0 = BPT * threadIdx.x;
        int32_t c[BPT], sum = 0;
        #pragma unroll
        for (int j = 0; j < BPT; ++j) {
            c[j] = 0;
            #pragma unroll
            for (int v = 0; v < kWaves; ++v) c[j] += wcnt[v][b0 + j];
            sum += c[j];
        }
        const int32_t incl = wave_incl_scan(sum);
        if (lane == 63) wtot[wave] = incl;
        __syncthreads();
        int32_t ex = incl - sum;
        for (int v = 0; v < wave; ++v) ex += wtot[v];
        #pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = b0 + j;
            lstart[b] = ex;
            int32_t run = ex;
            #pragma unroll
            for (int v = 0; v < kWaves; ++v) {
                const int32_t a = wcnt[v][b];
                wcnt[v][b] = run;
                run += a;
            }
            gbase[b] = base + bstart[seg * NB + b] + cnt[(int64_t)tile * NB + b];
            ex += c[j];
        }
    }
    __syncthreads();
    #pragma unroll
    for (int q = 0; q < kSsRounds; ++q) {
        if (bk[q] >= 0) {
            const int off = cw[bk[q]] + rk[q];
            skey[off] = kr[q];
            sval[off] = wbase + q * 64 + lane - base;
            sbk[off] = (Id)bk[q];
        }
    }
    __syncthreads();
    const int n_tile = (end - start) < kSsTile ? (end - start) : kSsTile;
    for (int q = threadIdx.x; q < n_tile; q += kSsThreads) {
        const int b = sbk[q];
        const int dst = gbase[b] + (q - lstart[b]);
        kout[dst] = skey[q];
        vout[dst] = sval[q];
    }
}

__device__ __forceinline__ uint64_t load_coherent(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t load_coherent(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup per (segment, bucket slot): the bucketed keys (kin, vin) of
// the bucket, sorted stably, into (kout, vout) at the same offsets.
template <int NB>
__global__ __launch_bounds__(kSsLocalThreads) void k_ss_local(SortSegs S, const int32_t* __restrict__ nspl,
                                                              const int32_t* __restrict__ bstart,
                                                              const int32_t* __restrict__ btot,
                                                              uint64_t* __restrict__ kin, int32_t* __restrict__ vin,
                                                              uint64_t* __restrict__ kout,
                                                              int32_t* __restrict__ vout)
{
    constexpr int kWaves = kSsLocalThreads / 64;
    __shared__ SsBlockLds L;
    __shared__ int32_t gb[256];
    const int seg = blockIdx.x / NB, b = blockIdx.x % NB;
    if (b > 2 * nspl[seg]) return;
    const int32_t size = btot[seg * NB + b];
    if (size == 0) return;
    const int64_t start = S.off[seg] + bstart[seg * NB + b];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((b & 1) || size == 1) {   // equal keys: already in order
        for (int32_t i = threadIdx.x; i < size; i += kSsLocalThreads) {
            kout[start + i] = kin[start + i];
            vout[start + i] = vin[start + i];
        }
        return;
    }
    uint64_t kr[kSsRounds];
    int32_t vr[kSsRounds];
    if (size <= kSsCap) {
        const int rounds = ss_rounds(size);
        #pragma unroll
        for (int q = 0; q < kSsRounds; ++q) {
            const int i = (wave * rounds + q) * 64 + lane;
            const bool in = q < rounds && i < size;
            kr[q] = in ? kin[start + i] : 0ull;
            vr[q] = in ? vin[start + i] : 0;
        }
        ss_block_sort(kr, vr, size, L);
        #pragma unroll
        for (int q = 0; q < kSsRounds; ++q) {
            const int i = (wave * rounds + q) * 64 + lane;
            if (q < rounds && i < size) { kout[start + i] = kr[q]; vout[start + i] = vr[q]; }
        }
        return;
    }
    // A bucket beyond the LDS: LSD passes through global memory, chunk by
    // chunk (kSsCap keys, kSsRounds rounds per wave) in order, between
    // (kin, vin) and (kout, vout); a chunk's keys are written straight to
    // their places.  Data written by an earlier pass is read with
    // cache-coherent loads.
    int dg[kSsRounds], rk[kSsRounds];
    uint64_t kmin = ~0ull, kmax = 0ull;
    for (int32_t c0 = 0; c0 < size; c0 += kSsCap) {
        const int nv = size - c0 < kSsCap ? size - c0 : kSsCap;
        #pragma unroll
        for (int q = 0; q < kSsRounds; ++q) {
            const int i = (wave * kSsRounds + q) * 64 + lane;
            kr[q] = i < nv ? kin[start + c0 + i] : 0ull;
        }
        uint64_t lo, hi;
        ss_key_range(kr, kSsRounds, nv, L.red, lo, hi);
        kmin = lo < kmin ? lo : kmin;
        kmax = hi > kmax ? hi : kmax;
    }
    const uint64_t diff = kmin ^ kmax;
    const int passes = diff ? (64 - __clzll((long long)diff) + 7) / 8 : 0;
    uint64_t* ks = kin; int32_t* vs = vin; uint64_t* kd = kout; int32_t* vd = vout;
    for (int p = 0; p < passes; ++p) {
        // digit totals over the bucket
        for (int i = threadIdx.x; i < kWaves * 256; i += kSsLocalThreads) (&L.wcnt[0][0])[i] = 0;
        __syncthreads();
        for (int32_t c0 = 0; c0 < size; c0 += kSsCap) {
            const int nv = size - c0 < kSsCap ? size - c0 : kSsCap;
            #pragma unroll
            for (int q = 0; q < kSsRounds; ++q) {
                const int i = (wave * kSsRounds + q) * 64 + lane;
                kr[q] = i < nv ? load_coherent(ks + start + c0 + i) : 0ull;
            }
            ss_rank_digits(kr, 8 * p, kSsRounds, nv, L.wcnt, dg, rk);   // wcnt accumulates over the chunks
        }
        __syncthreads();
        {
            int32_t c = 0;
            #pragma unroll
            for (int v = 0; v < kWaves; ++v) c += L.wcnt[v][threadIdx.x];
            const int32_t incl = wave_incl_scan(c);
            if (lane == 63) L.wtot[wave] = incl;
            __syncthreads();
            int32_t ex = incl - c;
            for (int v = 0; v < wave; ++v) ex += L.wtot[v];
            gb[threadIdx.x] = ex;   // the digit's next free place in the bucket
        }
        __syncthreads();
        for (int32_t c0 = 0; c0 < size; c0 += kSsCap) {
            const int nv = size - c0 < kSsCap ? size - c0 : kSsCap;
            #pragma unroll
            for (int q = 0; q < kSsRounds; ++q) {
                const int i = (wave * kSsRounds + q) * 64 + lane;
                kr[q] = i < nv ? load_coherent(ks + start + c0 + i) : 0ull;
                vr[q] = i < nv ? load_coherent(vs + start + c0 + i) : 0;
            }
            for (int i = threadIdx.x; i < kWaves * 256; i += kSsLocalThreads) (&L.wcnt[0][0])[i] = 0;
            __syncthreads();
            ss_rank_digits(kr, 8 * p, kSsRounds, nv, L.wcnt, dg, rk);
            __syncthreads();
            const int32_t c = ss_digit_starts(L.wcnt, 0, L.wtot);   // chunk-local starts
            __syncthreads();
            #pragma unroll
            for (int q = 0; q < kSsRounds; ++q) {
                if (dg[q] >= 0) {
                    // the digit's next free place + the key's offset among the chunk's keys of that digit
                    const int32_t dst = gb[dg[q]] + (L.wcnt[wave][dg[q]] + rk[q]) - L.wcnt[0][dg[q]];
                    kd[start + dst] = kr[q];
                    vd[start + dst] = vr[q];
                }
            }
            __syncthreads();
            gb[threadIdx.x] += c;
            __syncthreads();
        }
        uint64_t* tk = ks; ks = kd; kd = tk;
        int32_t* tv = vs; vs = vd; vd = tv;
    }
    if (ks != kout) {   // an even number of passes: the result is still in (kin, vin)
        for (int32_t i = threadIdx.x; i < size; i += kSsLocalThreads) {
            kout[start + i] = load_coherent(kin + start + i);
            vout[start + i] = load_coherent(vin + start + i);
        }
    }
}

// ---------------------------------------------------------------------------
// Staircases of the local region (the product decided exactly):
//   K[j]  = #{k : omega_j r_k <= z}   (rows; K is nonincreasing in j)
//   Jc[k] = #{j : omega_j r_k <= z}   (columns; Jc is nonincreasing in k)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool exact_le(double a, double b, double z)
{
    dd p = two_prod(a, b);
    if (p.hi < z) return true;
    if (p.hi > z) return false;
    return p.lo <= 0.0;
}

// One wave per 64 consecutive queries.  The queries are sorted, so the counts
// are nonincreasing along the wave: the counts of the wave's first and last
// queries come first, each from a 32-ary search by one half of the wave (32
// probes per step split the range into 33 parts), then every lane finishes
// with a binary search inside that bracket (a few steps where the sorted
// points are spread evenly).
__device__ __forceinline__ void staircase_body(const double* __restrict__ sorted, int32_t len,
                                               const double* __restrict__ q, int32_t nq, double z,
                                               int32_t* __restrict__ out, int32_t bid)
{
    const int lane = threadIdx.x & 63;
    const int32_t j0 = (int32_t)((bid * blockDim.x + threadIdx.x) & ~63u);
    if (j0 >= nq) return;                              // the whole wave
    const int32_t jl = j0 + 63 < nq ? j0 + 63 : nq - 1;
    const int half = lane >> 5, hl = lane & 31;
    const double wt = q[half ? jl : j0];
    // the count (first index whose product exceeds z) lies in [lo, hi]
    int32_t lo = 0, hi = len;
    while (hi - lo > 32) {
        const int64_t span = hi - lo;
        const int32_t pos = lo + (int32_t)(((int64_t)(hl + 1) * span) / 33);   // lo < pos < hi
        const uint64_t b = __ballot(exact_le(wt, sorted[pos], z));
        const int c = __popc(half ? (uint32_t)(b >> 32) : (uint32_t)b);        // probes at or below z
        const int32_t nlo = c > 0 ? lo + (int32_t)(((int64_t)c * span) / 33) + 1 : lo;
        const int32_t nhi = c < 32 ? lo + (int32_t)(((int64_t)(c + 1) * span) / 33) : hi;
        lo = nlo;
        hi = nhi;
    }
    {
        const int32_t pos = lo + hl;
        const uint64_t b = __ballot(pos < hi && exact_le(wt, sorted[pos], z));
        lo += __popc(half ? (uint32_t)(b >> 32) : (uint32_t)b);
    }
    const int32_t top = __shfl(lo, 0), bottom = __shfl(lo, 32);
    const int32_t j = j0 + lane;
    if (j > jl) return;
    const double w = q[j];
    lo = bottom;
    hi = top;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (exact_le(w, sorted[mid], z)) lo = mid + 1; else hi = mid;
    }
    out[j] = lo;
}

// Both staircases of a geometry in one launch (they are independent): the
// first nba workgroups count, for each sorted frequency, the sorted points
// whose product with it is at most z (K); the rest count, for each sorted
// point, the sorted frequencies (Jc).  One launch fewer on the plan's path.
__global__ __launch_bounds__(256) void k_staircase(const double* __restrict__ rs, int32_t n,
                                                   const double* __restrict__ ws, int32_t m, double z,
                                                   int32_t* __restrict__ K, int32_t* __restrict__ Jc, int32_t nba)
{
    if ((int32_t)blockIdx.x < nba) staircase_body(rs, n, ws, m, z, K, blockIdx.x);
    else staircase_body(ws, m, rs, n, z, Jc, blockIdx.x - nba);
}

// ---------------------------------------------------------------------------
// Alg. 1 (Subdivide), level by level in one 256-thread block.  Every mixed
// block of a level becomes a Node; its split follows the quasi-optimal
// SplitIndices of Sec. 4.1 (candidate rows equispaced over the rows that hold
// a local entry, minimal mixed area, ties to the smaller row).  Numbering is
// deterministic: nodes in level order, children in (parent, position) order.
// ---------------------------------------------------------------------------
// The split of one mixed node (Alg. 1) and the classes of its children.
struct NodeSplit {
    int32_t js, ks;
    bool cl, ca, ur_m, ur_d, ll_m, ll_d;
};

// Candidate counts up to this are evaluated with all their loads in flight.
constexpr int32_t kSplitUnroll = 16;

// kj1 = K[R.j1], kj0 = K[R.j0], jc = Jc[R.k0], loaded by the caller.
__device__ __forceinline__ NodeSplit split_node(const Rect& R, int32_t kj1, int32_t kj0, int32_t jc,
                                                const int32_t* __restrict__ K, int64_t min_size, int32_t ncand)
{
    NodeSplit o;
    int32_t js = 0, ks = 0;
    if (kj1 >= R.k1 + 1) {              // wholly local
        js = R.j1; ks = R.k1;
    } else if (kj0 <= R.k0) {           // wholly asymptotic
        js = R.j0 - 1; ks = R.k0 - 1;
    } else {
        // the last row holding a local entry: K[j] > k0 <=> j < Jc[k0]
        int32_t jl = jc - 1;
        if (jl > R.j1) jl = R.j1;
        int64_t best = INT64_MAX;
        int32_t span = jl - R.j0;
        // more candidates than rows is every row (the exact optimum)
        int32_t nc = span > 0 ? (ncand <= span ? ncand : span + 1) : 1;
        // candidate c is row j0 + floor(c span / (nc - 1)); the quotient is
        // formed in double, exactly: c span < 2^53, and a non-integer quotient
        // is at least 1/(nc-1) away from an integer
        auto row_of = [&](int32_t c) {
            if (nc == span + 1) return R.j0 + c;            // every row
            return span > 0 ? R.j0 + (int32_t)floor((double)c * (double)span / (double)(nc - 1)) : R.j0;
        };
        auto consider = [&](int32_t j, int32_t kraw) {
            int32_t k = kraw - 1;
            if (k > R.k1) k = R.k1;
            if (k < R.k0) k = R.k0 - 1;
            int64_t mixed = (int64_t)(j - R.j0 + 1) * (R.k1 - k) + (int64_t)(R.j1 - j) * (k - R.k0 + 1);
            if (mixed < best) { best = mixed; js = j; ks = k; }
        };
        if (nc <= kSplitUnroll) {
            // all candidate loads in flight together, then taken in order
            int32_t jv[kSplitUnroll], kv[kSplitUnroll];
            #pragma unroll
            for (int32_t c = 0; c < kSplitUnroll; ++c) {
                jv[c] = row_of(c < nc ? c : 0);
                kv[c] = K[jv[c]];
            }
            #pragma unroll
            for (int32_t c = 0; c < kSplitUnroll; ++c)
                if (c < nc) consider(jv[c], kv[c]);
        } else {
            // batches of kSplitUnroll candidates with their loads in flight
            for (int32_t c0 = 0; c0 < nc; c0 += kSplitUnroll) {
                int32_t jv[kSplitUnroll], kv[kSplitUnroll];
                #pragma unroll
                for (int32_t c = 0; c < kSplitUnroll; ++c) {
                    jv[c] = row_of(c0 + c < nc ? c0 + c : c0);
                    kv[c] = K[jv[c]];
                }
                #pragma unroll
                for (int32_t c = 0; c < kSplitUnroll; ++c)
                    if (c0 + c < nc) consider(jv[c], kv[c]);
            }
        }
    }
    o.js = js; o.ks = ks;
    o.cl = ks >= R.k0 && js >= R.j0;
    o.ca = js < R.j1 && ks < R.k1;
    o.ur_m = o.ur_d = o.ll_m = o.ll_d = false;
    if (ks < R.k1 && js >= R.j0) {
        if ((int64_t)(js - R.j0 + 1) * (R.k1 - ks) > min_size) o.ur_m = true; else o.ur_d = true;
    }
    if (js < R.j1 && ks >= R.k0) {
        if ((int64_t)(R.j1 - js) * (ks - R.k0 + 1) > min_size) o.ll_m = true; else o.ll_d = true;
    }
    return o;
}

// Nodes per thread per pass.  (Several per thread serialise their candidate
// loads within the thread, and a pass waits for its slowest thread: one is
// faster.)
constexpr int kSubNpt = 1;
// One workgroup does the whole subdivision.  256 threads rather than 1024:
// a 1024-thread workgroup needs a compute unit with sixteen free wave slots,
// which the execution running beside the plan rarely leaves.
constexpr int kSubThreads = 256;
// The first entries of each level's queue live in LDS (the queue of the next
// level is written while the current one is read, so two buffers); entries
// past them go to the global queues at the same index.
constexpr int kSubLds = 1920;

__global__ __launch_bounds__(kSubThreads) void k_subdivide(const int32_t* __restrict__ K, const int32_t* __restrict__ Jc,
                                                    int32_t m, int32_t n, int64_t min_size, int32_t ncand, Arena A,
                                                    Summary* __restrict__ sum, const int32_t* __restrict__ errs,
                                                    int32_t n_errs)
{
    __shared__ int32_t wsum[4][16];
    __shared__ Rect lq[2][kSubLds];
    int tid = threadIdx.x;
    // the summary starts clear (this is the first planning kernel to use it),
    // with the input check's verdict
    int bad = 0;
    for (int32_t i = tid; i < n_errs; i += kSubThreads) bad |= errs[i];
    bad = __syncthreads_or(bad);
    if (tid == 0) {
        *sum = Summary{};
        sum->domain_error = bad ? 1 : 0;
    }
    Rect* cur = A.q0;
    Rect* nxt = A.q1;
    int cb = 0;                                      // LDS buffer of the current level
    int32_t n_cur = (m > 0 && n > 0) ? 1 : 0;
    if (tid == 0 && n_cur) lq[0][0] = Rect{0, m - 1, 0, n - 1};
    int32_t n_nodes = 0, n_l = 0, n_a = 0, n_d = 0;
    int32_t overflow = 0;
    int32_t level = 0;
    __syncthreads();
    while (n_cur > 0) {
        ++level;
        int32_t n_next = 0;
        for (int32_t c0 = 0; c0 < n_cur; c0 += kSubThreads * kSubNpt) {
            const int32_t i0 = c0 + tid * kSubNpt;
            Rect R[kSubNpt];
            NodeSplit S[kSubNpt];
            int32_t cnt[4] = {0, 0, 0, 0};
            int32_t kj1[kSubNpt], kj0[kSubNpt], jc[kSubNpt];
            #pragma unroll
            for (int q = 0; q < kSubNpt; ++q) {
                bool act = i0 + q < n_cur;
                R[q] = act ? (i0 + q < kSubLds ? lq[cb][i0 + q] : cur[i0 + q]) : Rect{0, 0, 0, 0};
            }
            #pragma unroll
            for (int q = 0; q < kSubNpt; ++q) {   // all header loads in flight together
                kj1[q] = K[R[q].j1];
                kj0[q] = K[R[q].j0];
                jc[q] = Jc[R[q].k0];
            }
            #pragma unroll
            for (int q = 0; q < kSubNpt; ++q) {
                bool act = i0 + q < n_cur;
                if (act) {
                    S[q] = split_node(R[q], kj1[q], kj0[q], jc[q], K, min_size, ncand);
                    cnt[0] += S[q].cl;
                    cnt[1] += S[q].ca;
                    cnt[2] += (int)S[q].ur_d + (int)S[q].ll_d;
                    cnt[3] += (int)S[q].ur_m + (int)S[q].ll_m;
                }
            }
            int32_t v[4] = {cnt[0], cnt[1], cnt[2], cnt[3]};
            int32_t tot[4];
            block_scan<int32_t, 4, kSubThreads / 64>(v, tot, wsum);
            int32_t l_slot = n_l + v[0], a_slot = n_a + v[1], d_slot = n_d + v[2], m_slot = n_next + v[3];
            const int32_t next_base = n_nodes + n_cur;   // first node index of the next level
            #pragma unroll
            for (int q = 0; q < kSubNpt; ++q) {
                if (i0 + q >= n_cur) continue;
                const Rect& Rq = R[q];
                const NodeSplit& o = S[q];
                int32_t node = n_nodes + i0 + q;
                Node nd;
                nd.j0 = Rq.j0; nd.j1 = Rq.j1; nd.k0 = Rq.k0; nd.k1 = Rq.k1;
                nd.js = o.js; nd.ks = o.ks;
                nd.lblk = o.cl ? l_slot : -1;
                nd.ablk = o.ca ? a_slot : -1;
                nd.level = level; nd.pad = 0;
                nd.ur = -1; nd.ll = -1;
                if (o.ur_m) {
                    const Rect c = Rect{Rq.j0, o.js, o.ks + 1, Rq.k1};
                    if (m_slot < kSubLds) lq[cb ^ 1][m_slot] = c;
                    else if (m_slot < A.q_cap) nxt[m_slot] = c;
                    nd.ur = next_base + m_slot;
                    ++m_slot;
                }
                if (o.ur_d) { if (d_slot < A.d_cap) A.db[d_slot] = DBlock{Rq.j0, o.js, o.ks + 1, Rq.k1}; nd.ur = encode_direct(d_slot); ++d_slot; }
                if (o.ll_m) {
                    const Rect c = Rect{o.js + 1, Rq.j1, Rq.k0, o.ks};
                    if (m_slot < kSubLds) lq[cb ^ 1][m_slot] = c;
                    else if (m_slot < A.q_cap) nxt[m_slot] = c;
                    nd.ll = next_base + m_slot;
                    ++m_slot;
                }
                if (o.ll_d) { if (d_slot < A.d_cap) A.db[d_slot] = DBlock{o.js + 1, Rq.j1, Rq.k0, o.ks}; nd.ll = encode_direct(d_slot); ++d_slot; }
                if (node < A.node_cap) A.nodes[node] = nd;
                if (o.cl) {
                    if (l_slot < A.l_cap) {
                        LBlock b;
                        b.j0 = Rq.j0; b.j1 = o.js; b.k0 = Rq.k0; b.k1 = o.ks;
                        b.R = 0.0; b.item0 = 0; b.nitems = 0; b.level = level; b.pad = 0;
                        A.lb[l_slot] = b;
                    }
                    ++l_slot;
                }
                if (o.ca) {
                    if (a_slot < A.a_cap) {
                        ABlock b = {};
                        b.j0 = o.js + 1; b.j1 = Rq.j1; b.k0 = o.ks + 1; b.k1 = Rq.k1; b.level = level;
                        A.ab[a_slot] = b;
                    }
                    ++a_slot;
                }
            }
            n_l += tot[0];
            n_a += tot[1];
            n_d += tot[2];
            n_next += tot[3];
        }
        n_nodes += n_cur;
        if (n_next > A.q_cap || n_nodes > A.node_cap) {
            overflow = 1;
            n_next = n_next > A.q_cap ? A.q_cap : n_next;
        }
        if (level >= kMaxLevels) overflow = 2;
        Rect* t = cur; cur = nxt; nxt = t;
        cb ^= 1;
        n_cur = overflow ? 0 : n_next;
        __syncthreads();
    }
    if (overflow != 2 && (n_l > A.l_cap || n_a > A.a_cap || n_d > A.d_cap)) overflow = 1;
    if (tid == 0) {
        sum->n_nodes = n_nodes; sum->n_l = n_l; sum->n_a = n_a; sum->n_d = n_d;
        sum->levels = level; sum->overflow = overflow;
    }
}

// ---------------------------------------------------------------------------
// Per-block parameters (grid-stride over the blocks the subdivision made).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t iceil(double x) { return (int32_t)ceil(x); }

__global__ void k_block_params(PlanDev P, Arena A, int32_t dft_max, double sigma, Summary* __restrict__ sum)
{
    if (sum->overflow) return;
    const int32_t n_l = sum->n_l, n_a = sum->n_a;
    const int w = P.w;
    const int32_t nb = n_l > n_a ? n_l : n_a;
    for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        if (b < n_a) {
            ABlock B = A.ab[b];
            double rlo = P.rs[B.k0], rhi = P.rs[B.k1];
            double wlo = P.ws[B.j0], whi = P.ws[B.j1];
            double C = 0.5 * (rlo + rhi);
            double X = fmax(rhi - C, C - rlo);
            double D = 0.5 * (wlo + whi);
            double S = fmax(whi - D, D - wlo);
            if (!(S > 1e-280)) S = 1e-280;
            // grid spacing: the largest power of two with S h <= pi / sigma
            double h = exp2(floor(log2(kPi / (sigma * S))));
            if (S * h > kPi / sigma) h *= 0.5;
            double span = X / h;
            if (!(span < (double)(1 << (kMaxFftLog2 - 3)))) {   // grid too large for the FFT sizes
                atomicOr(&sum->grid_error, 1);
                span = 0.0;
            }
            int32_t llo = iceil(-span - 0.5 * w) - 1;
            int32_t lhi = iceil(span - 0.5 * w) + w;
            int32_t N1 = lhi - llo + 1;
            B.C = C; B.D = D; B.h = h; B.r0 = rlo; B.alpha = 0.5 * w * h;
            B.llo = llo; B.N1 = N1;
            int32_t fft = (dft_max >= 0 && N1 <= dft_max) ? 0 : 1;
            int32_t N2 = 0;
            if (fft) {
                int32_t maxl = llo < 0 ? -llo : llo;
                if (lhi > maxl) maxl = lhi;
                N2 = 64;
                while (N2 < 4 * maxl + 4) N2 <<= 1;
                // h N2 / (2 pi): exact scaling of the double-double 1/(2 pi)
                B.Khi = h * (double)N2 * kInvTwoPi;
                B.Klo = h * (double)N2 * kInvTwoPiLo;
            }
            B.fft = fft; B.N2 = N2;
            int32_t ncol = B.k1 - B.k0 + 1;
            B.nitems = (ncol + P.spread_chunk - 1) / P.spread_chunk;
            A.ab[b] = B;
        }
        if (b < n_l) {
            LBlock L = A.lb[b];
            double R = P.rs[L.k1];
            if (R == 0.0) {
                double wm = P.ws[L.j1];
                R = wm > 0.0 ? P.z / wm : 1.0;
            }
            L.R = R;
            int32_t ncol = L.k1 - L.k0 + 1;
            L.nitems = (ncol + kLocalChunk - 1) / kLocalChunk;
            A.lb[b] = L;
        }
    }
}

// ---------------------------------------------------------------------------
// Offsets and totals (one workgroup): exclusive scans over the blocks of item
// counts and grid slots, the FFT size classes, membership statistics.
// The block and item scans run as one workgroup of kPlanScanThreads (at most
// 128 VGPRs per wave): a workgroup this small fits on a compute unit as soon
// as one workgroup of a running transform's kernels retires there, where a
// 1024-thread one waits for a whole compute unit to drain.
// ---------------------------------------------------------------------------
constexpr int kPlanScanThreads = 256;

__global__ __launch_bounds__(kPlanScanThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_plan_scan(PlanDev P, Arena A, Summary* __restrict__ sum)
{
    __shared__ int64_t wsum[2][16];
    __shared__ int32_t cls_cnt[kMaxFftLog2 + 1];
    __shared__ int32_t cls_first[kMaxFftLog2 + 1];
    __shared__ long long red[9][kPlanScanThreads / 64];
    if (sum->overflow) return;
    const int32_t n_l = sum->n_l, n_a = sum->n_a, n_d = sum->n_d;
    int tid = threadIdx.x;
    const int nch = P.nch;
    if (tid <= kMaxFftLog2) cls_cnt[tid] = 0;
    __syncthreads();
    // membership statistics: rows / columns of local and asymptotic blocks,
    // direct entries, grid cells and FFT points, and the row-side work of the
    // asymptotic blocks (rows x cells on the direct-sum path, rows on the FFT
    // path), gathered in the same passes
    constexpr int kStats = 9;
    long long st[kStats] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    constexpr int kVpt = 8;                          // blocks per thread per pass (2048 per pass)
    int64_t l_items = 0;
    for (int32_t c0 = 0; c0 < n_l; c0 += kPlanScanThreads * kVpt) {
        const int32_t i0 = c0 + tid * kVpt;
        int64_t v[kVpt][1];
        #pragma unroll
        for (int k = 0; k < kVpt; ++k) {
            v[k][0] = 0;
            if (i0 + k < n_l) {
                const LBlock L = A.lb[i0 + k];
                v[k][0] = L.nitems;
                st[0] += L.j1 - L.j0 + 1;
                st[1] += L.k1 - L.k0 + 1;
            }
        }
        int64_t tot[1];
        block_scan_vpt<1, kVpt, kPlanScanThreads / 64>(v, tot, wsum);
        #pragma unroll
        for (int k = 0; k < kVpt; ++k)
            if (i0 + k < n_l) A.lb[i0 + k].item0 = (int32_t)(l_items + v[k][0]);
        l_items += tot[0];
    }
    int64_t a_items = 0, grid = 0;
    for (int32_t c0 = 0; c0 < n_a; c0 += kPlanScanThreads * kVpt) {
        const int32_t i0 = c0 + tid * kVpt;
        int64_t v[kVpt][2];
        bool fft[kVpt];
        int32_t n2[kVpt];
        #pragma unroll
        for (int k = 0; k < kVpt; ++k) {
            v[k][0] = v[k][1] = 0;
            fft[k] = false;
            n2[k] = 0;
            if (i0 + k < n_a) {
                const ABlock B = A.ab[i0 + k];
                v[k][0] = B.nitems;
                v[k][1] = B.fft ? (int64_t)B.N2 : (int64_t)B.N1;
                fft[k] = B.fft != 0;
                n2[k] = B.N2;
                const long long rows = B.j1 - B.j0 + 1;
                st[2] += rows;
                st[3] += B.k1 - B.k0 + 1;
                if (B.fft) { st[6] += B.N2; st[8] += rows; }
                else { st[5] += B.N1; st[7] += rows * B.N1; }
            }
        }
        int64_t tot[2];
        block_scan_vpt<2, kVpt, kPlanScanThreads / 64>(v, tot, wsum);
        #pragma unroll
        for (int k = 0; k < kVpt; ++k) {
            const int32_t i = i0 + k;
            if (i < n_a) {
                A.ab[i].item0 = (int32_t)(a_items + v[k][0]);
                A.ab[i].grid_off = (grid + v[k][1]) * nch;
                A.gslot[i] = grid + v[k][1];
                if (fft[k]) atomicAdd(&cls_cnt[31 - __clz(n2[k])], 1);
            }
        }
        a_items += tot[0];
        grid += tot[1];
    }
    if (tid == 0) A.gslot[n_a] = grid;
    __syncthreads();
    if (tid == 0) {
        int32_t f = 0;
        for (int c = 0; c <= kMaxFftLog2; ++c) {
            cls_first[c] = f;
            sum->fft_first[c] = f;
            sum->fft_count[c] = cls_cnt[c];
            f += cls_cnt[c];
            cls_cnt[c] = 0;
        }
        sum->n_fft = f;
    }
    __syncthreads();
    // FFT-path blocks grouped by size class (order inside a class is immaterial)
    for (int32_t i = tid; i < n_a; i += kPlanScanThreads) {
        ABlock B = A.ab[i];
        if (B.fft) {
            int c = 31 - __clz(B.N2);
            int32_t slot = cls_first[c] + atomicAdd(&cls_cnt[c], 1);
            A.fft_list[slot] = i;
            A.ab[i].fft_slot = slot;
        }
    }
    for (int32_t i = tid; i < n_d; i += kPlanScanThreads) {
        DBlock Db = A.db[i];
        st[4] += (long long)(Db.j1 - Db.j0 + 1) * (Db.k1 - Db.k0 + 1);
    }
    for (int q = 0; q < kStats; ++q) {
        long long x = st[q];
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
        if ((tid & 63) == 0) red[q][tid >> 6] = x;
    }
    __syncthreads();
    if (tid == 0) {
        long long t[kStats] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int q = 0; q < kStats; ++q)
            for (int w2 = 0; w2 < kPlanScanThreads / 64; ++w2) t[q] += red[q][w2];
        sum->l_row = t[0]; sum->l_col = t[1]; sum->a_row = t[2]; sum->a_col = t[3];
        sum->d_ent = t[4]; sum->dft_cells = t[5]; sum->fft_points = t[6];
        sum->dft_row_cells = t[7]; sum->fft_rows = t[8];
        sum->n_litems = (int32_t)l_items; sum->n_aitems = (int32_t)a_items;
        sum->max_nch = nch;
        sum->grid_cells = grid;
        if (l_items > A.litem_cap || a_items > A.aitem_cap) sum->overflow = 1;
    }
}

// ---------------------------------------------------------------------------
// Work items (grid-stride over all items: local first, then asymptotic).
// An item is a chunk of one block's columns; an asymptotic item also carries
// the subgrid of cells its points can reach (one cell of margin each side).
// ---------------------------------------------------------------------------
__global__ void k_items(PlanDev P, Arena A, Summary* __restrict__ sum, int32_t* __restrict__ a_cells)
{
    if (sum->overflow) return;
    const int32_t n_l = sum->n_l, n_a = sum->n_a;
    const int32_t n_li = sum->n_litems, n_ai = sum->n_aitems;
    const int w = P.w;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_li + n_ai; i += gridDim.x * blockDim.x) {
        if (i < n_li) {
            int32_t lo = 0, hi = n_l - 1;             // last block with item0 <= i
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (A.lb[mid].item0 <= i) lo = mid; else hi = mid - 1;
            }
            const LBlock L = A.lb[lo];
            int32_t it = i - L.item0;
            int32_t ka = L.k0 + it * kLocalChunk;
            int32_t kb = ka + kLocalChunk;
            if (kb > L.k1 + 1) kb = L.k1 + 1;
            Item I;
            I.blk = lo; I.ka = ka; I.kb = kb; I.sub_lo = 0; I.sub_n = 0; I.dense = 0; I.off = 0;
            A.litems[i] = I;
        } else {
            int32_t ia = i - n_li;
            int32_t lo = 0, hi = n_a - 1;
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (A.ab[mid].item0 <= ia) lo = mid; else hi = mid - 1;
            }
            const ABlock B = A.ab[lo];
            int32_t it = ia - B.item0;
            int32_t ka = B.k0 + it * P.spread_chunk;
            int32_t kb = ka + P.spread_chunk - 1;
            if (kb > B.k1) kb = B.k1;
            int32_t lhi = B.llo + B.N1 - 1;
            double u0 = (P.rs[ka] - B.C) / B.h, u1 = (P.rs[kb] - B.C) / B.h;
            int32_t s0 = iceil(u0 - 0.5 * w) - 1;
            int32_t s1 = iceil(u1 - 0.5 * w) + w;
            if (s0 < B.llo) s0 = B.llo;
            if (s1 > lhi) s1 = lhi;
            Item I;
            I.blk = lo; I.ka = ka; I.kb = kb + 1; I.sub_lo = s0; I.sub_n = s1 - s0 + 1; I.off = 0;
            // first cells of the points lie in s0 .. s1 - w + 1 (one cell of
            // margin each side for rounding): dense if at most kSpreadAnchors,
            // medium if at most kSpreadAnchorsMed
            const int32_t anchors = I.sub_n - w + 1;
            I.dense = !P.mfma ? 0
                    : anchors <= kSpreadAnchors ? 1
                    : (anchors <= kSpreadAnchorsMed && P.nch <= kMfmaMedMaxChannels) ? 2 : 0;
            A.aitems[ia] = I;
            a_cells[ia] = I.sub_n;
        }
    }
}

// Partial-subgrid offsets of the asymptotic items, and the spreading order:
// dense items at alist[0 ..), medium ones after them, and the others at
// alist[n_ai - 1], alist[n_ai - 2], ..., each list in item order (one
// workgroup).
__global__ __launch_bounds__(kPlanScanThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_item_scan(
    PlanDev P, Arena A, Summary* __restrict__ sum, const int32_t* __restrict__ a_cells)
{
    __shared__ int64_t wsum[3][16];
    __shared__ int32_t n_dense_total;
    if (sum->overflow) return;
    const int32_t n_ai = sum->n_aitems;
    const int nch = P.nch;
    constexpr int kVpt = 8;                          // items per thread per pass (2048 per pass)
    // the dense items' total first: the medium ones follow them in the list
    {
        int32_t nd = 0;
        for (int32_t i = threadIdx.x; i < n_ai; i += kPlanScanThreads) nd += A.aitems[i].dense == 1 ? 1 : 0;
        for (int o = 32; o >= 1; o >>= 1) nd += __shfl_xor(nd, o);
        if (threadIdx.x == 0) n_dense_total = 0;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) atomicAdd(&n_dense_total, nd);
        __syncthreads();
    }
    const int64_t nd_total = n_dense_total;
    int64_t run = 0, run_dense = 0, run_med = 0;
    for (int32_t c0 = 0; c0 < n_ai; c0 += kPlanScanThreads * kVpt) {
        const int32_t i0 = c0 + threadIdx.x * kVpt;
        int64_t v[kVpt][3];
        int cls[kVpt];
        #pragma unroll
        for (int k = 0; k < kVpt; ++k) {
            const bool act = i0 + k < n_ai;
            v[k][0] = act ? (int64_t)a_cells[i0 + k] : 0;
            cls[k] = act ? A.aitems[i0 + k].dense : 0;
            v[k][1] = cls[k] == 1 ? 1 : 0;
            v[k][2] = cls[k] == 2 ? 1 : 0;
        }
        int64_t tot[3];
        block_scan_vpt<3, kVpt, kPlanScanThreads / 64>(v, tot, wsum);
        #pragma unroll
        for (int k = 0; k < kVpt; ++k) {
            const int32_t i = i0 + k;
            if (i < n_ai) {
                A.aitems[i].off = (run + v[k][0]) * nch;
                // dense from the front, then medium, the others from the back
                const int64_t nd_before = run_dense + v[k][1], nm_before = run_med + v[k][2];
                const int64_t pos = cls[k] == 1 ? nd_before
                                  : cls[k] == 2 ? nd_total + nm_before
                                                : n_ai - 1 - (i - nd_before - nm_before);
                A.alist[pos] = i;
            }
        }
        run += tot[0];
        run_dense += tot[1];
        run_med += tot[2];
    }
    if (threadIdx.x == 0) {
        sum->part_cells = run;
        sum->n_adense = (int32_t)run_dense;
        sum->n_amed = (int32_t)run_med;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

static SortSegs sort_segs(int32_t na, int32_t nb)
{
    SortSegs S;
    S.off[0] = 0; S.off[1] = na; S.off[2] = na + nb;
    const int ta = cdiv(na, kSortTile), tb = cdiv(nb, kSortTile);
    S.tile0[0] = 0; S.tile0[1] = ta; S.tile0[2] = ta + tb;
    S.hoff[0] = 0; S.hoff[1] = 256 * ta; S.hoff[2] = 256 * (ta + tb);
    return S;
}

// The 1024-slot splitter sort is taken up to 2^18 keys: measured faster than
// the LSD sort there (200000 keys: plan 0.263 against 0.287 ms); at 1e6 its
// sample and bucket sorts (ballot ranking, LDS round trips per round) cost
// 342 us of GPU time against the LSD sort's 276.
constexpr int32_t kSsLargeMax = 1 << 18;
static_assert(kSsLargeMax <= SsCfg<1024>::kMaxLen, "splitter sort capacity");

enum class SortPath { small, splitter64, splitter1024, lsd };

static SortPath sort_path(int32_t na, int32_t nb)
{
    const int32_t mx = na > nb ? na : nb;
    if (mx <= kSsCap) return SortPath::small;
    if (mx <= SsCfg<64>::kMaxLen) return SortPath::splitter64;
    if (mx <= kSsLargeMax) return SortPath::splitter1024;
    return SortPath::lsd;
}

static SortSegs ss_segs(int32_t na, int32_t nb)
{
    SortSegs S;
    S.off[0] = 0; S.off[1] = na; S.off[2] = na + nb;
    const int ta = cdiv(na, kSsTile), tb = cdiv(nb, kSsTile);
    S.tile0[0] = 0; S.tile0[1] = ta; S.tile0[2] = ta + tb;
    S.hoff[0] = S.hoff[1] = S.hoff[2] = 0;
    return S;
}

template <int NB>
static hipError_t launch_splitter_sort(const double* r, int32_t na, const double* w, int32_t nb, uint64_t* k0,
                                       int32_t* v0, uint64_t* k1, int32_t* v1, int32_t* hist, int32_t* errs,
                                       hipStream_t s)
{
    using C = SsCfg<NB>;
    const SortSegs S = ss_segs(na, nb);
    const int tiles = S.tile0[2];
    uint64_t* spl = (uint64_t*)hist;
    int32_t* nspl = hist + C::kNsplOff;
    int32_t* bstart = hist + C::kStartOff;
    int32_t* btot = hist + C::kTotOff;
    int32_t* cnt = hist + C::kCntOff;
    hipLaunchKernelGGL(k_ss_sample<NB>, dim3(2), dim3(1024), 0, s, r, w, S, spl, nspl);
    hipLaunchKernelGGL(k_ss_count<NB>, dim3(tiles), dim3(kSsThreads), 0, s, r, w, S, spl, nspl, cnt, errs);
    hipLaunchKernelGGL(k_ss_scan<NB>, dim3(2), dim3(NB), 0, s, S, cnt, bstart, btot);
    hipLaunchKernelGGL(k_ss_scatter<NB>, dim3(tiles), dim3(kSsThreads), 0, s, r, w, S, spl, nspl, cnt, bstart, k1,
                       v1);
    hipLaunchKernelGGL(k_ss_local<NB>, dim3(2 * NB), dim3(kSsLocalThreads), 0, s, S, nspl, bstart, btot, k1, v1,
                       k0, v0);
    return hipGetLastError();
}

hipError_t launch_keys_and_sort(const double* r, int32_t na, const double* w, int32_t nb, uint64_t* k0, int32_t* v0,
                                uint64_t* k1, int32_t* v1, int32_t* hist, int32_t* errs, hipStream_t s)
{
    const SortPath path = sort_path(na, nb);
    if (path == SortPath::small) {
        if (na + nb == 0) return hipSuccess;
        const SortSegs S = ss_segs(na, nb);
        hipLaunchKernelGGL(k_sort_small, dim3(2), dim3(kSsLocalThreads), 0, s, r, w, S, k0, v0, errs);
        return hipGetLastError();
    }
    if (path == SortPath::splitter64) return launch_splitter_sort<64>(r, na, w, nb, k0, v0, k1, v1, hist, errs, s);
    if (path == SortPath::splitter1024)
        return launch_splitter_sort<1024>(r, na, w, nb, k0, v0, k1, v1, hist, errs, s);
    const SortSegs S = sort_segs(na, nb);
    const int tiles = S.tile0[2];
    if (tiles == 0) return hipSuccess;
    // the per-tile counts, then the 2 x 256 digit totals
    int32_t* dtot = hist + S.hoff[2];
    hipLaunchKernelGGL(k_make_keys, dim3(tiles), dim3(kSortThreads), 0, s, r, w, S, k0, v0, hist, errs);
    uint64_t* kin = k0; int32_t* vin = v0; uint64_t* kout = k1; int32_t* vout = v1;
    for (int pass = 0; pass < 8; ++pass) {
        if (pass > 0)   // the first pass's counts come with the keys
            hipLaunchKernelGGL(k_sort_hist, dim3(tiles), dim3(kSortThreads), 0, s, kin, S, 8 * pass, hist);
        hipLaunchKernelGGL(k_sort_scan, dim3(2 * 256 / 4), dim3(256), 0, s, hist, dtot, S);
        hipLaunchKernelGGL(k_sort_scatter, dim3(tiles), dim3(kSortThreads), 0, s, kin, vin, kout, vout, S, 8 * pass,
                           hist, dtot);
        uint64_t* tk = kin; kin = kout; kout = tk;
        int32_t* tv = vin; vin = vout; vout = tv;
    }
    return hipGetLastError();   // eight passes: the result is back in (k0, v0)
}

hipError_t launch_reduce_errs(const int32_t* errs, int32_t n, int32_t* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_errs, dim3(1), dim3(256), 0, s, errs, n, flag);
    return hipGetLastError();
}

int sort_tiles(int32_t na, int32_t nb)
{
    switch (sort_path(na, nb)) {
        case SortPath::small: return 2;
        case SortPath::splitter64:
        case SortPath::splitter1024: return cdiv(na, kSsTile) + cdiv(nb, kSsTile);
        default: return cdiv(na, kSortTile) + cdiv(nb, kSortTile);
    }
}

int sort_hist_len(int32_t na, int32_t nb)
{
    switch (sort_path(na, nb)) {
        case SortPath::small: return 1;
        case SortPath::splitter64: return SsCfg<64>::kCntOff + 64 * sort_tiles(na, nb);
        case SortPath::splitter1024: return SsCfg<1024>::kCntOff + 1024 * sort_tiles(na, nb);
        default: return 256 * sort_tiles(na, nb) + 2 * 256;
    }
}

hipError_t launch_planning(const PlanDev& P, const Arena& A, int32_t* K, int32_t* Jc, int32_t* a_cells,
                           int64_t min_size, int32_t ncand, int32_t dft_max, double sigma, Summary* sum,
                           const int32_t* errs, int32_t n_errs, hipStream_t s)
{
    const int32_t n = P.n, m = P.m;
    hipLaunchKernelGGL(k_staircase, dim3(cdiv(m, 256) + cdiv(n, 256)), dim3(256), 0, s, P.rs, n, P.ws, m, P.z, K,
                       Jc, cdiv(m, 256));
    hipLaunchKernelGGL(k_subdivide, dim3(1), dim3(kSubThreads), 0, s, K, Jc, m, n, min_size, ncand, A, sum, errs, n_errs);
    hipLaunchKernelGGL(k_block_params, dim3(256), dim3(128), 0, s, P, A, dft_max, sigma, sum);
    hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(kPlanScanThreads), 0, s, P, A, sum);
    hipLaunchKernelGGL(k_items, dim3(512), dim3(128), 0, s, P, A, sum, a_cells);
    hipLaunchKernelGGL(k_item_scan, dim3(1), dim3(kPlanScanThreads), 0, s, P, A, sum, a_cells);
    return hipGetLastError();
}

}  // namespace nuht
