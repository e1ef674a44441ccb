// Counting-sort binning of particles into a uniform grid of square bins.
//
// The Delaunay step of App. B needs, for every mesh node, the particles near
// it.  Instead of a global triangulation (the paper used CGAL, App. A), the
// particles are sorted by bin so that every bin row segment is a contiguous
// range of a sorted position array.  Four kernels:
//   1. count:   key and in-bin rank per particle (atomic histogram);
//   2. scan:    exclusive prefix sum of the histogram (three-phase);
//   3. scatter: sorted positions and the sorted -> user permutation;
//   4. fix:     per-bin insertion sort by user id, so the sorted order equals
//               a stable sort by key (bitwise deterministic).
#include "kernels.h"

namespace p2m {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__global__ void __launch_bounds__(256) k_bin_count(const double2* __restrict__ pos, int N,
                                                   const SetDesc* __restrict__ sets, int S, uint32_t nbins,
                                                   uint32_t* __restrict__ key, int32_t* __restrict__ rank,
                                                   int32_t* __restrict__ count,
                                                   unsigned long long* __restrict__ diag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SetDesc& sd = sets[set_search(S, i, [&](int s) { return sets[s].p0; })];
    const MeshD m = sd.m;
    const Grid g = sd.g;
    const double2 p = pos[i];
    const double x1 = add_rn(m.x0, mul_rn(static_cast<double>(m.nx), m.H));
    const double y1 = add_rn(m.y0, mul_rn(static_cast<double>(m.ny), m.H));
    uint32_t k;
    // NaN fails every comparison, so it is caught here as well.
    if (p.x >= m.x0 && p.x <= x1 && p.y >= m.y0 && p.y <= y1) {
        int bx = static_cast<int>(floor((p.x - g.x0) / g.bw));
        int by = static_cast<int>(floor((p.y - g.y0) / g.bw));
        bx = min(max(bx, 0), g.nbx - 1);
        by = min(max(by, 0), g.nby - 1);
        k = static_cast<uint32_t>(sd.b0) + static_cast<uint32_t>(by) * static_cast<uint32_t>(g.nbx) +
            static_cast<uint32_t>(bx);
    } else {
        k = nbins;
        atomicAdd(&diag[D_BAD], 1ull);
    }
    key[i] = k;
    rank[i] = atomicAdd(&count[k], 1);
}

// Phase 1 of the scan: per-tile exclusive scan, tile totals to tsum.
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tile(const int32_t* __restrict__ in,
                                                            int32_t* __restrict__ out, int n,
                                                            int32_t* __restrict__ tsum) {
    __shared__ int32_t s[SCAN_THREADS];
    const int t = threadIdx.x;
    const int base = blockIdx.x * SCAN_TILE + t * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int idx = base + k;
        v[k] = idx < n ? in[idx] : 0;
        sum += v[k];
    }
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        const int32_t add = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    int32_t run = s[t] - sum;  // exclusive prefix of this thread within the tile
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int idx = base + k;
        if (idx < n) out[idx] = run;
        run += v[k];
    }
    if (t == SCAN_THREADS - 1) tsum[blockIdx.x] = s[t];
}

// Phase 2: exclusive scan of the tile totals (one block); tsum[ntiles] = total.
__global__ void __launch_bounds__(1024) k_scan_sums(int32_t* __restrict__ tsum, int ntiles) {
    __shared__ int32_t s[1024];
    __shared__ int32_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < ntiles; base += 1024) {
        const int idx = base + t;
        const int32_t v = idx < ntiles ? tsum[idx] : 0;
        s[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t add = t >= off ? s[t - off] : 0;
            __syncthreads();
            s[t] += add;
            __syncthreads();
        }
        const int32_t c = carry;
        if (idx < ntiles) tsum[idx] = c + s[t] - v;
        __syncthreads();
        if (t == 1023) carry = c + s[t];
        __syncthreads();
    }
    if (t == 0) tsum[ntiles] = carry;
}

// Phase 3: add tile offsets; out[n] = total.
__global__ void __launch_bounds__(256) k_scan_add(int32_t* __restrict__ out, int n,
                                                  const int32_t* __restrict__ tsum, int ntiles) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tsum[i / SCAN_TILE];
    if (i == n) out[n] = tsum[ntiles];
}

__global__ void __launch_bounds__(256) k_bin_scatter(const double2* __restrict__ pos, int N,
                                                     const uint32_t* __restrict__ key,
                                                     const int32_t* __restrict__ rank,
                                                     const int32_t* __restrict__ start,
                                                     double2* __restrict__ pos_s,
                                                     int32_t* __restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int slot = start[key[i]] + rank[i];
    pos_s[slot] = pos[i];
    perm[slot] = i;
}

// Bins hold O(1) particles at the intended bin width; insertion sort is fine
// and keeps the result independent of the atomic arrival order.
__global__ void __launch_bounds__(256) k_bin_fix(const int32_t* __restrict__ start, int nbins,
                                                 double2* __restrict__ pos_s, int32_t* __restrict__ perm,
                                                 unsigned long long* __restrict__ diag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    const int s = start[b], e = start[b + 1];
    for (int i = s + 1; i < e; ++i) {
        const int32_t pi = perm[i];
        const double2 xi = pos_s[i];
        int j = i - 1;
        while (j >= s && perm[j] > pi) {
            perm[j + 1] = perm[j];
            pos_s[j + 1] = pos_s[j];
            --j;
        }
        perm[j + 1] = pi;
        pos_s[j + 1] = xi;
    }
    // coincident particles always share a bin: no Delaunay triangulation
    int dup = 0;
    for (int i = s + 1; i < e; ++i) {
        const double2 a = pos_s[i];
        for (int k = s; k < i; ++k) {
            const double2 b = pos_s[k];
            dup += (a.x == b.x && a.y == b.y) ? 1 : 0;
        }
    }
    if (dup) atomicAdd(&diag[D_DUP], static_cast<unsigned long long>(dup));
}

inline int blocks_for(int64_t n, int threads) { return static_cast<int>((n + threads - 1) / threads); }

}  // namespace

int64_t scan_tile_count(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

int exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tsum, hipStream_t st) {
    const int ntiles = static_cast<int>(scan_tile_count(n));
    k_scan_tile<<<ntiles, SCAN_THREADS, 0, st>>>(in, out, static_cast<int>(n), tsum);
    k_scan_sums<<<1, 1024, 0, st>>>(tsum, ntiles);
    k_scan_add<<<blocks_for(n + 1, 256), 256, 0, st>>>(out, static_cast<int>(n), tsum, ntiles);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int bin_particles(const BinBuffers& b, const double* pos, int64_t N, const SetDesc* sets, int S, int64_t nbins,
                  unsigned long long* diag, hipStream_t st) {
    PhaseTimer _timer(PH_BIN, st);
    // count[0..nbins] (the last entry collects invalid particles)
    int rc = fill_i32(b.count, 0, nbins + 1, st);
    if (rc) return rc;
    k_bin_count<<<blocks_for(N, 256), 256, 0, st>>>(reinterpret_cast<const double2*>(pos), static_cast<int>(N),
                                                    sets, S, static_cast<uint32_t>(nbins), b.key, b.rank,
                                                    b.count, diag);
    P2M_HIP(hipGetLastError());
    rc = exclusive_scan(b.count, b.start, nbins + 1, b.tsum, st);
    if (rc) return rc;
    k_bin_scatter<<<blocks_for(N, 256), 256, 0, st>>>(reinterpret_cast<const double2*>(pos), static_cast<int>(N),
                                                      b.key, b.rank, b.start,
                                                      reinterpret_cast<double2*>(b.pos_s), b.perm);
    k_bin_fix<<<blocks_for(nbins, 256), 256, 0, st>>>(b.start, static_cast<int>(nbins),
                                                      reinterpret_cast<double2*>(b.pos_s), b.perm, diag);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
