// Counting-sort binning of particles into a uniform grid of square bins.
//
// The Delaunay step of App. B needs, for every mesh node, the particles near
// it.  Instead of a global triangulation (the paper used CGAL, App. A), the
// particles are sorted by bin so that every bin row segment is a contiguous
// range of a sorted position array.  The sort is a two-level counting sort
// without global atomics; bins are grouped into super-bins of 2^SBS
// consecutive bin keys (rows of bins):
//   1. key:   bin key per particle, and per chunk of particles an LDS
//             histogram over super-bins;
//   2. scan:  exclusive prefix sums of the (super-bin, chunk) histogram
//             within tiles, and the tile totals (their prefix is formed by
//             the consumers); this kernel also clears the diagnostics;
//   3. part:  each chunk scatters (position, key, user id) into its super-bin
//             ranges (runs of consecutive slots per chunk);
//   4. local: one block per super-bin counts its bins in LDS, writes their
//             start offsets, places its particles, and sorts each bin by user
//             id, so the sorted order equals a stable sort by key (bitwise
//             deterministic, independent of atomic arrival order).
// Four launches in all: each dependent launch costs microseconds by itself.
#include <mutex>

#include "kernels.h"

namespace p2m {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr int BT = 1024;         // threads of the binning kernels (16 waves)
constexpr int MAX_SB = 8192;     // super-bins (LDS counters of kernels 1 and 3)
constexpr int MAX_SBS = 14;      // bins per super-bin <= 2^14 (LDS of kernel 4)

// Bin key of particle i (key nbins: outside its set's mesh, or non-finite).
__device__ __forceinline__ uint32_t bin_key(const double2 p, const SetDesc& sd, uint32_t nbins) {
    const MeshD m = sd.m;
    const Grid g = sd.g;
    const double x1 = add_rn(m.x0, mul_rn(static_cast<double>(m.nx), m.H));
    const double y1 = add_rn(m.y0, mul_rn(static_cast<double>(m.ny), m.H));
    // NaN fails every comparison, so it is caught here as well.
    if (!(p.x >= m.x0 && p.x <= x1 && p.y >= m.y0 && p.y <= y1)) return nbins;
    int bx = static_cast<int>(floor((p.x - g.x0) / g.bw));
    int by = static_cast<int>(floor((p.y - g.y0) / g.bw));
    bx = min(max(bx, 0), g.nbx - 1);
    by = min(max(by, 0), g.nby - 1);
    return static_cast<uint32_t>(sd.b0) + static_cast<uint32_t>(by) * static_cast<uint32_t>(g.nbx) +
           static_cast<uint32_t>(bx);
}

struct BinGeom {
    int64_t N;
    uint32_t nbins;
    int nch;       // chunks of particles (one block each in kernels 1 and 3)
    int64_t cs;    // particles per chunk
    int sbs;       // log2(bins per super-bin)
    int nsb;       // super-bins
};

// Exclusive prefix of v over the block (NT threads, all active) and the
// block total in *total: shuffle scans within each wave, one pass over the
// wave totals in LDS (two barriers; wsum holds NT / 64 entries).
template <int NT = BT>
__device__ __forceinline__ int block_exclusive_prefix(int v, int32_t* wsum, int* total = nullptr) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int before = 0, all = 0;
    for (int k = 0; k < NT / 64; ++k) {
        const int t = wsum[k];
        before += k < w ? t : 0;
        all += t;
    }
    __syncthreads();  // wsum may be reused after this
    if (total) *total = all;
    return before + inc - v;
}

// Exclusive scan of in[0..n) into out (n <= a few entries per thread).
__device__ __forceinline__ void block_exclusive_scan(const int32_t* in, int32_t* out, int n, int32_t* wsum) {
    const int per = (n + BT - 1) / BT;
    const int r0 = threadIdx.x * per;
    int acc = 0;
    for (int k = 0; k < per; ++k)
        if (r0 + k < n) acc += in[r0 + k];
    int run = block_exclusive_prefix(acc, wsum);
    for (int k = 0; k < per; ++k)
        if (r0 + k < n) {
            out[r0 + k] = run;
            run += in[r0 + k];
        }
    __syncthreads();
}

// 1. keys and the (super-bin, chunk) histogram, super-bin major
__global__ void __launch_bounds__(BT) k_bin_key(const double2* __restrict__ pos, const SetDesc* __restrict__ sets,
                                               int S, BinGeom bg, uint32_t* __restrict__ key,
                                               int32_t* __restrict__ hist) {
    __shared__ int32_t lh[MAX_SB];
    const int c = blockIdx.x;
    for (int k = threadIdx.x; k < bg.nsb; k += BT) lh[k] = 0;
    __syncthreads();
    const int64_t lo = c * bg.cs, hi = min(bg.N, lo + bg.cs);
#pragma unroll 4
    for (int64_t i = lo + threadIdx.x; i < hi; i += BT) {
        const SetDesc& sd = sets[set_search(S, i, [&](int s) { return sets[s].p0; })];
        const uint32_t k = bin_key(pos[i], sd, bg.nbins);
        key[i] = k;
        atomicAdd(&lh[k >> bg.sbs], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < bg.nsb; k += BT) hist[static_cast<int64_t>(k) * bg.nch + c] = lh[k];
}

// 2. exclusive scan of hist[0..n) within tiles of SCAN_TILE entries (entry n,
// the end offset, scans a zero), tile totals to tsum; block 0 clears the
// diagnostics (nothing before this kernel counts into them).
__global__ void __launch_bounds__(SCAN_THREADS) k_hist_scan(int32_t* __restrict__ hist, int n,
                                                            int32_t* __restrict__ tsum,
                                                            unsigned long long* __restrict__ diag) {
    __shared__ int32_t wsum[SCAN_THREADS / 64];
    const int t = threadIdx.x;
    if (blockIdx.x == 0 && t < D_COUNT) diag[t] = 0ull;
    const int base = blockIdx.x * SCAN_TILE + t * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int idx = base + k;
        v[k] = idx < n ? hist[idx] : 0;
        sum += v[k];
    }
    int total = 0;
    int32_t run = block_exclusive_prefix<SCAN_THREADS>(sum, wsum, &total);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int idx = base + k;
        if (idx <= n) hist[idx] = run;
        run += v[k];
    }
    if (t == 0) tsum[blockIdx.x] = total;
}

// Global exclusive offset of histogram entry i: its tile-local prefix plus
// the totals of the tiles before it (tpre: their exclusive prefix in LDS).
__device__ __forceinline__ int hist_offset(const int32_t* hist, const int32_t* tpre, int64_t i) {
    return hist[i] + tpre[i / SCAN_TILE];
}

// 3. each chunk scatters its particles into its slots of every super-bin.
// A sub-chunk of `sub` particles is first ordered by super-bin in LDS, so that
// consecutive threads write consecutive slots of each run (coalesced).
// Dynamic LDS: gcur[nsb], lcnt[nsb], lstart[nsb], then sub (position, key,
// user id) records.
// PPT records per thread: sub <= PPT * BT.  Consecutive slots of a run are
// written together only if a sub-chunk holds several particles of each
// super-bin, so many super-bins (large grids) take the larger sub-chunks.
template <int PPT>
__global__ void __launch_bounds__(BT) k_bin_part(const double2* __restrict__ pos, const uint32_t* __restrict__ key,
                                                BinGeom bg, const int32_t* __restrict__ offs,
                                                const int32_t* __restrict__ tsum, int ntiles, int sub,
                                                double2* __restrict__ part_pos, uint32_t* __restrict__ part_key,
                                                int32_t* __restrict__ part_uid) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t part[BT / 64];
    const int nsb = bg.nsb;
    double2* spos = reinterpret_cast<double2*>(smem);
    uint32_t* skey = reinterpret_cast<uint32_t*>(spos + sub);
    int32_t* suid = reinterpret_cast<int32_t*>(skey + sub);
    int32_t* gcur = suid + sub;
    int32_t* lcnt = gcur + nsb;
    int32_t* lstart = lcnt + nsb;
    int32_t* tpre = lstart + nsb;  // [ntiles]
    const int c = blockIdx.x;
    block_exclusive_scan(tsum, tpre, ntiles, part);
    for (int k = threadIdx.x; k < nsb; k += BT) gcur[k] = hist_offset(offs, tpre, static_cast<int64_t>(k) * bg.nch + c);
    const int64_t lo = c * bg.cs, hi = min(bg.N, lo + bg.cs);
    for (int64_t b0 = lo; b0 < hi; b0 += sub) {
        const int n = static_cast<int>(min<int64_t>(sub, hi - b0));
        for (int k = threadIdx.x; k < nsb; k += BT) lcnt[k] = 0;
        __syncthreads();
        // loads at clamped indices (n >= 1), so that the staging arrays stay
        // in registers; only real elements are counted and placed
        // (coordinates as plain doubles: an array of the vector type would be
        // kept in scratch memory across the scan)
        uint32_t kk[PPT];
        int rr[PPT];
        double px[PPT], py[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int e = min(static_cast<int>(threadIdx.x) + j * BT, n - 1);
            kk[j] = key[b0 + e];
            const double2 p = pos[b0 + e];
            px[j] = p.x;
            py[j] = p.y;
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int e = threadIdx.x + j * BT;
            rr[j] = e < n ? atomicAdd(&lcnt[kk[j] >> bg.sbs], 1) : 0;
        }
        __syncthreads();
        block_exclusive_scan(lcnt, lstart, nsb, part);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int e = threadIdx.x + j * BT;
            if (e < n) {
                const int sl = lstart[kk[j] >> bg.sbs] + rr[j];
                spos[sl] = make_double2(px[j], py[j]);
                skey[sl] = kk[j];
                suid[sl] = static_cast<int32_t>(b0 + e);
            }
        }
        __syncthreads();
        for (int sl = threadIdx.x; sl < n; sl += BT) {
            const uint32_t k = skey[sl];
            const int sb = static_cast<int>(k >> bg.sbs);
            const int slot = gcur[sb] + (sl - lstart[sb]);
            part_pos[slot] = spos[sl];
            part_key[slot] = k;
            part_uid[slot] = suid[sl];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nsb; k += BT) gcur[k] += lcnt[k];
        __syncthreads();
    }
}

// 4. one block per super-bin: bin counts and start offsets, placement, and a
// per-bin sort by user id (bins hold O(1) particles at the intended width).
// When the super-bin's particles fit (`cap`), they are staged in LDS and
// placed and sorted there, and the sorted run is written once, coalesced;
// otherwise the ranks go through global memory and the bins are sorted in
// place.  Dynamic LDS: positions [cap], user ids [cap], bin starts [M + 1],
// then 16-bit keys, ranks and output order [cap] each.
__global__ void __launch_bounds__(BT) k_bin_local(BinGeom bg, const int32_t* __restrict__ offs,
                                                 const int32_t* __restrict__ tsum, int cap,
                                                 const double2* __restrict__ part_pos,
                                                 const uint32_t* __restrict__ part_key,
                                                 const int32_t* __restrict__ part_uid, int32_t* __restrict__ rank,
                                                 int32_t* __restrict__ start, double2* __restrict__ pos_s,
                                                 int32_t* __restrict__ perm, unsigned long long* __restrict__ diag) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t wsum[BT / 64];
    __shared__ int32_t ndup;
    const int M = 1 << bg.sbs;
    double2* lpos = reinterpret_cast<double2*>(smem);
    int32_t* luid = reinterpret_cast<int32_t*>(lpos + cap);
    int32_t* pre = luid + cap;
    uint16_t* lkey = reinterpret_cast<uint16_t*>(pre + M + 1);
    uint16_t* lrank = lkey + cap;
    uint16_t* lord = lrank + cap;
    const int b = blockIdx.x;
    // the super-bin's range: tile-local offsets plus the totals of the tiles
    // before them
    int lo, hi;
    {
        const int64_t ilo = static_cast<int64_t>(b) * bg.nch, ihi = static_cast<int64_t>(b + 1) * bg.nch;
        const int tlo = static_cast<int>(ilo / SCAN_TILE), thi = static_cast<int>(ihi / SCAN_TILE);
        int slo = 0, shi = 0;
        for (int k = threadIdx.x; k < thi; k += BT) {
            const int v = tsum[k];
            slo += k < tlo ? v : 0;
            shi += v;
        }
        int tot_lo = 0, tot_hi = 0;
        (void)block_exclusive_prefix(slo, wsum, &tot_lo);
        (void)block_exclusive_prefix(shi, wsum, &tot_hi);
        lo = offs[ilo] + tot_lo;
        hi = offs[ihi] + tot_hi;
    }
    const int n = hi - lo;
    const bool staged = n <= cap;
    const uint32_t k0 = static_cast<uint32_t>(b) << bg.sbs;
    for (int k = threadIdx.x; k <= M; k += BT) pre[k] = 0;
    if (threadIdx.x == 0) ndup = 0;
    __syncthreads();
    // counts (pre[k + 1] collects bin k) and each particle's rank in its bin
    if (staged) {
        for (int e = threadIdx.x; e < n; e += BT) {
            const int k = static_cast<int>(part_key[lo + e] - k0);
            lkey[e] = static_cast<uint16_t>(k);
            lpos[e] = part_pos[lo + e];
            luid[e] = part_uid[lo + e];
            lrank[e] = static_cast<uint16_t>(atomicAdd(&pre[k + 1], 1));
        }
    } else {
#pragma unroll 4
        for (int e = lo + threadIdx.x; e < hi; e += BT) rank[e] = atomicAdd(&pre[part_key[e] - k0 + 1], 1);
    }
    __syncthreads();
    // inclusive scan of pre[1..M]: thread t sums a run of M / BT entries
    {
        const int run = M / BT;
        const int r0 = 1 + threadIdx.x * run;
        int acc = 0;
        for (int k = 0; k < run; ++k) acc += pre[r0 + k];
        int base = block_exclusive_prefix(acc, wsum);
        for (int k = 0; k < run; ++k) {
            base += pre[r0 + k];
            pre[r0 + k] = base;
        }
    }
    __syncthreads();
    // start offsets of this super-bin's bins (and of the excluded bucket)
    for (int k = threadIdx.x; k < M; k += BT) {
        const uint32_t gk = k0 + static_cast<uint32_t>(k);
        if (gk <= bg.nbins) start[gk] = lo + pre[k];
    }
    if (k0 <= bg.nbins && bg.nbins < k0 + static_cast<uint32_t>(M) && threadIdx.x == 0) {
        start[bg.nbins + 1] = static_cast<int32_t>(bg.N);
        // particles outside their mesh (or non-finite) make up the excluded bucket
        diag[D_BAD] = static_cast<unsigned long long>(bg.N - (lo + pre[bg.nbins - k0]));
    }
    int dup = 0;
    if (staged) {
        for (int e = threadIdx.x; e < n; e += BT) lord[pre[lkey[e]] + lrank[e]] = static_cast<uint16_t>(e);
        __syncthreads();
        // per bin: insertion sort by user id; coincident particles always
        // share a bin, so pairs of them are counted here
        for (int k = threadIdx.x; k < M; k += BT) {
            if (k0 + static_cast<uint32_t>(k) >= bg.nbins) break;  // the excluded bucket is not sorted
            const int s0 = pre[k], s1 = pre[k + 1];
            for (int i = s0 + 1; i < s1; ++i) {
                const uint16_t oi = lord[i];
                const int32_t ui = luid[oi];
                int j = i - 1;
                while (j >= s0 && luid[lord[j]] > ui) {
                    lord[j + 1] = lord[j];
                    --j;
                }
                lord[j + 1] = oi;
            }
            for (int i = s0 + 1; i < s1; ++i) {
                const double2 pa = lpos[lord[i]];
                for (int q = s0; q < i; ++q) {
                    const double2 pc = lpos[lord[q]];
                    dup += (pa.x == pc.x && pa.y == pc.y) ? 1 : 0;
                }
            }
        }
        __syncthreads();
        for (int d = threadIdx.x; d < n; d += BT) {
            const int e = lord[d];
            pos_s[lo + d] = lpos[e];
            perm[lo + d] = luid[e];
        }
    } else {
        // placement
#pragma unroll 4
        for (int e = lo + threadIdx.x; e < hi; e += BT) {
            const int slot = lo + pre[part_key[e] - k0] + rank[e];
            pos_s[slot] = part_pos[e];
            perm[slot] = part_uid[e];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < M; k += BT) {
            if (k0 + static_cast<uint32_t>(k) >= bg.nbins) break;  // the excluded bucket is not sorted
            const int s0 = lo + pre[k], s1 = lo + pre[k + 1];
            for (int i = s0 + 1; i < s1; ++i) {
                const int32_t pi = perm[i];
                const double2 xi = pos_s[i];
                int j = i - 1;
                while (j >= s0 && perm[j] > pi) {
                    perm[j + 1] = perm[j];
                    pos_s[j + 1] = pos_s[j];
                    --j;
                }
                perm[j + 1] = pi;
                pos_s[j + 1] = xi;
            }
            for (int i = s0 + 1; i < s1; ++i) {
                const double2 pa = pos_s[i];
                for (int q = s0; q < i; ++q) {
                    const double2 pc = pos_s[q];
                    dup += (pa.x == pc.x && pa.y == pc.y) ? 1 : 0;
                }
            }
        }
    }
    if (dup) atomicAdd(&ndup, dup);
    __syncthreads();
    if (threadIdx.x == 0 && ndup) atomicAdd(&diag[D_DUP], static_cast<unsigned long long>(ndup));
}

inline int blocks_for(int64_t n, int threads) { return static_cast<int>((n + threads - 1) / threads); }

}  // namespace

int64_t scan_tile_count(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

int bin_layout(int64_t N, int64_t nbins, int* nch, int* sbs, int* nsb) {
    int shift = 12;
    while (shift < MAX_SBS && (nbins >> shift) + 1 > MAX_SB) ++shift;
    if ((nbins >> shift) + 1 > MAX_SB) {
        set_error("binning grid too large (%lld bins)", static_cast<long long>(nbins));
        return P2M_EINVAL;
    }
    *sbs = shift;
    *nsb = static_cast<int>((nbins >> shift) + 1);
    *nch = static_cast<int>(std::min<int64_t>(256, std::max<int64_t>(1, (N + 4095) / 4096)));
    return P2M_OK;
}

int bin_particles(const BinBuffers& b, const double* pos, int64_t N, const SetDesc* sets, int S, int64_t nbins,
                  unsigned long long* diag, hipStream_t st) {
    PhaseTimer _timer(PH_BIN, st);
    BinGeom bg;
    int rc = bin_layout(N, nbins, &bg.nch, &bg.sbs, &bg.nsb);
    if (rc) return rc;
    bg.N = N;
    bg.nbins = static_cast<uint32_t>(nbins);
    bg.cs = (N + bg.nch - 1) / bg.nch;
    const int64_t nh = static_cast<int64_t>(bg.nsb) * bg.nch;
    const double2* P = reinterpret_cast<const double2*>(pos);
    k_bin_key<<<bg.nch, BT, 0, st>>>(P, sets, S, bg, b.key, b.hist);
    const int ntiles = static_cast<int>(scan_tile_count(nh + 1));
    k_hist_scan<<<ntiles, SCAN_THREADS, 0, st>>>(b.hist, static_cast<int>(nh), b.tsum, diag);
    // dynamic LDS beyond 64 KB must be allowed once per function
    constexpr int64_t LDS_MAX = 163840 - 2048;
    static std::once_flag lds_once;
    static hipError_t lds_err = hipSuccess;
    std::call_once(lds_once, [] {
        lds_err = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bin_local),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX);
        if (lds_err == hipSuccess)
            lds_err = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bin_part<4>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX);
    });
    P2M_HIP(lds_err);
    // sub-chunk size: four records per thread in up to 160 KB (as many as
    // fit beside the counters) when a chunk holds more than two per thread
    // or the super-bins outnumber the threads: the partition runs one block
    // per CU, so the LDS costs no occupancy, and a whole chunk in one pass
    // saves a round of barriers and scans; else two per thread in 64 KB
    const int64_t fixed = 12 * static_cast<int64_t>(bg.nsb) + 4 * static_cast<int64_t>(ntiles);
    const bool wide = bg.nsb > BT || bg.cs > 2 * BT;
    int sub = (wide ? 4 : 2) * BT;
    const int64_t lds_cap = wide ? LDS_MAX : 65536;
    while (sub > 256 && fixed + 24 * static_cast<int64_t>(sub) > lds_cap) sub >>= 1;
    if (fixed + 24 * static_cast<int64_t>(sub) > lds_cap) {
        set_error("binning: too many super-bins (%d)", bg.nsb);
        return P2M_EINVAL;
    }
    const size_t lds = static_cast<size_t>(24) * sub + static_cast<size_t>(fixed);
    if (wide)
        k_bin_part<4><<<bg.nch, BT, lds, st>>>(P, b.key, bg, b.hist, b.tsum, ntiles, sub,
                                               reinterpret_cast<double2*>(b.part_pos), b.part_key, b.part_uid);
    else
        k_bin_part<2><<<bg.nch, BT, lds, st>>>(P, b.key, bg, b.hist, b.tsum, ntiles, sub,
                                               reinterpret_cast<double2*>(b.part_pos), b.part_key, b.part_uid);
    // particles of a super-bin staged in LDS: as many as fit beside the bin
    // starts in 160 KB (16-byte position, user id, three 16-bit fields)
    const int M = 1 << bg.sbs;
    const int64_t room = LDS_MAX - 4 * static_cast<int64_t>(M + 1);
    const int cap = static_cast<int>(std::min<int64_t>(std::max<int64_t>(room / 26, 0) & ~int64_t(7), 65535));
    const size_t llds = static_cast<size_t>(cap) * 26 + 4 * static_cast<size_t>(M + 1);
    k_bin_local<<<bg.nsb, BT, llds, st>>>(bg, b.hist, b.tsum, cap, reinterpret_cast<const double2*>(b.part_pos), b.part_key,
                                          b.part_uid, b.rank, b.start, reinterpret_cast<double2*>(b.pos_s), b.perm,
                                          diag);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
