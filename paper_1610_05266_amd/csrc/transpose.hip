// Particle-major index of the weights' entries, and the two adjoint gathers
// it allows (handles built with P2M_DETERMINISTIC).
//
// The transpose of P2M (eq. p2m) sends d L / d mesh value of node i to every
// particle of the node's support, and the position adjoint of the weights
// (App. B) sends each entry's derivative to its particle.  Summed with
// atomics, the order of the additions depends on the schedule, so the bits
// of a gradient vary from run to run.  Here the entries are indexed by
// particle once per build (a counting sort by user id; each particle's
// entries then sorted by entry index), and each particle sums its own
// entries in that fixed order: no atomics on the results, the same bits on
// every run.
#include "kernels.h"

namespace p2m {

namespace {

constexpr int TB = 256;        // threads per block
constexpr int TSCAN = 2048;    // entries per block of the count scan
constexpr int TSCAN_PT = TSCAN / TB;

// Entry e of the grid over all entries: k = e / n_slots, slot = e % n_slots
// for e < KMAX n_slots (the ELL arrays), then the overflow rows' entries
// (k >= KMAX of the slots whose rows are long).  Writes the entry's user id,
// its node and its entry index; false when there is no such entry.  One
// thread per entry, so that the atomics of a row's entries run side by side
// instead of one after another.
__device__ __forceinline__ bool entry_of(const WeightsView& w, int64_t e, int32_t& u, int64_t& node, int64_t& ei) {
    const int64_t ns = w.n_slots;
    int64_t slot;
    int k;
    if (e < KMAX * ns) {
        k = static_cast<int>(e / ns);
        slot = e - k * ns;
    } else {
        // overflow entries are visited through their slot: e - KMAX ns runs
        // over (k - KMAX) * n_slots + slot
        const int64_t r = e - KMAX * ns;
        k = KMAX + static_cast<int>(r / ns);
        slot = r - (k - KMAX) * ns;
    }
    const uint32_t meta = w.meta[slot];
    const int n = row_len(meta);
    if (k >= n) return false;
    const SetDesc& sd = w.sets[set_search(w.S, slot / TILE_N, [&](int s) { return w.sets[s].t0; })];
    int i, j;
    if (!slot_ij(sd, slot, i, j)) return false;
    node = ij_node(sd, i, j);
    const int32_t orow = k >= KMAX ? w.orow[slot] : 0;
    u = k < KMAX ? w.idx[k * ns + slot] : w.oidx[ovf_at(w.n_ovf, orow, k)];
    ei = entry_at(ns, w.n_ovf, orow, slot, k);
    return true;
}

// Entries of the grid: every ELL entry, then (KROW - KMAX) per slot for the
// long rows (empty unless a row is long).
inline int64_t entry_grid(const WeightsView& w) { return static_cast<int64_t>(KROW) * w.n_slots; }

// 1. entries per particle
__global__ void __launch_bounds__(256) k_tcount(WeightsView w, int64_t ne, int32_t* __restrict__ cnt) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= ne) return;
    int32_t u;
    int64_t node, ei;
    if (entry_of(w, e, u, node, ei)) atomicAdd(&cnt[u], 1);
}

// Exclusive prefix of v over the block and the block total.
__device__ __forceinline__ int block_prefix(int v, int32_t* ws, int& total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
    }
    if (lane == 63) ws[wv] = inc;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < TB / 64; ++k) {
        before += k < wv ? ws[k] : 0;
        total += ws[k];
    }
    __syncthreads();
    return before + inc - v;
}

// 2a. tile-local exclusive prefix of cnt[0..n) into ptr, tile totals to tsum
__global__ void __launch_bounds__(TB) k_tscan_tiles(const int32_t* __restrict__ cnt, int64_t n,
                                                   int32_t* __restrict__ ptr, int32_t* __restrict__ tsum) {
    __shared__ int32_t ws[TB / 64];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * TSCAN + threadIdx.x * TSCAN_PT;
    int v[TSCAN_PT];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < TSCAN_PT; ++k) {
        v[k] = base + k < n ? cnt[base + k] : 0;
        sum += v[k];
    }
    int total;
    int run = block_prefix(sum, ws, total);
#pragma unroll
    for (int k = 0; k < TSCAN_PT; ++k) {
        if (base + k < n) ptr[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

// 2b. exclusive prefix of the tile totals (one block), the grand total in
// tsum[nt]
__global__ void __launch_bounds__(TB) k_tscan_totals(int32_t* __restrict__ tsum, int nt) {
    __shared__ int32_t ws[TB / 64];
    int carry = 0;
    for (int b0 = 0; b0 < nt; b0 += TB) {
        const int i = b0 + static_cast<int>(threadIdx.x);
        const int v = i < nt ? tsum[i] : 0;
        int total;
        const int ex = block_prefix(v, ws, total);
        if (i < nt) tsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tsum[nt] = carry;
}

// 2c. add the tile offsets; ptr[n] = the grand total; the counts become the
// fill cursors (zeroed)
__global__ void __launch_bounds__(TB) k_tscan_add(int32_t* __restrict__ ptr, int64_t n,
                                                 const int32_t* __restrict__ tsum, int nt,
                                                 int32_t* __restrict__ cnt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (i < n) {
        ptr[i] += tsum[i / TSCAN];
        cnt[i] = 0;
    }
    if (i == n) ptr[n] = tsum[nt];
}

// 3. every entry to its particle's range (order within a range: arrival)
__global__ void __launch_bounds__(TB) k_tfill(WeightsView w, int64_t ne, const int32_t* __restrict__ ptr,
                                             int32_t* __restrict__ cur, int32_t* __restrict__ ent,
                                             int32_t* __restrict__ nodes) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (e >= ne) return;
    int32_t u;
    int64_t node, ei;
    if (!entry_of(w, e, u, node, ei)) return;
    const int32_t at = ptr[u] + atomicAdd(&cur[u], 1);
    ent[at] = static_cast<int32_t>(ei);
    nodes[at] = static_cast<int32_t>(node);
}

// 4. each particle's range sorted by entry index (a handful of entries)
__global__ void __launch_bounds__(TB) k_tsort(const int32_t* __restrict__ ptr, int64_t N,
                                             int32_t* __restrict__ ent, int32_t* __restrict__ nodes) {
    const int64_t u = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (u >= N) return;
    const int32_t s0 = ptr[u], s1 = ptr[u + 1];
    for (int32_t i = s0 + 1; i < s1; ++i) {
        const int32_t e = ent[i], nd = nodes[i];
        int32_t j = i - 1;
        while (j >= s0 && ent[j] > e) {
            ent[j + 1] = ent[j];
            nodes[j + 1] = nodes[j];
            --j;
        }
        ent[j + 1] = e;
        nodes[j + 1] = nd;
    }
}

// P2M^t per particle: grad_vals[u][c] = sum over its entries (fixed order)
// of psi * grad_mesh[node][c], each product and sum in TG as the atomic form
// takes them.
template <typename TW, typename TG, int CC>
__global__ void __launch_bounds__(TB) k_project_bwd_gather(WeightsView w, const TW* __restrict__ wm,
                                                          const TW* __restrict__ wo, const TG* __restrict__ gmesh,
                                                          int Crt, TG* __restrict__ gvals) {
    constexpr int NC = CC > 0 ? CC : CMAX;
    const int C = CC > 0 ? CC : Crt;
    const int64_t u = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (u >= w.N) return;
    const int64_t split = KMAX * w.n_slots;
    TG acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = TG(0);
    const int32_t s1 = w.tptr[u + 1];
    for (int32_t p = w.tptr[u]; p < s1; ++p) {
        const int64_t e = w.tent[p];
        const int64_t node = w.tnode[p];
        const TG wk = static_cast<TG>(e < split ? wm[e] : wo[e - split]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < C) acc[c] += wk * gmesh[node * C + c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < C) gvals[u * C + c] = acc[c];
}

// grad_pos[u] += the sum of its entries' derivatives (fixed order)
__global__ void __launch_bounds__(TB) k_gpos_gather(WeightsView w, double2* __restrict__ gpos) {
    const int64_t u = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (u >= w.N) return;
    double sx = 0.0, sy = 0.0;
    const int32_t s1 = w.tptr[u + 1];
    for (int32_t p = w.tptr[u]; p < s1; ++p) {
        const double2 g = w.gent[w.tent[p]];
        sx += g.x;
        sy += g.y;
    }
    if (w.tptr[u] < s1) {
        double2 o = gpos[u];
        o.x += sx;
        o.y += sy;
        gpos[u] = o;
    }
}

inline unsigned grid(int64_t n) { return static_cast<unsigned>((n + TB - 1) / TB); }

template <typename TW, typename TG>
void launch_gather(const WeightsView& w, const TW* wm, const TW* wo, const void* gmesh, int C, void* gvals,
                   hipStream_t st) {
    const TG* g = static_cast<const TG*>(gmesh);
    TG* o = static_cast<TG*>(gvals);
    switch (C) {
        case 1: k_project_bwd_gather<TW, TG, 1><<<grid(w.N), TB, 0, st>>>(w, wm, wo, g, C, o); break;
        case 2: k_project_bwd_gather<TW, TG, 2><<<grid(w.N), TB, 0, st>>>(w, wm, wo, g, C, o); break;
        case 3: k_project_bwd_gather<TW, TG, 3><<<grid(w.N), TB, 0, st>>>(w, wm, wo, g, C, o); break;
        case 4: k_project_bwd_gather<TW, TG, 4><<<grid(w.N), TB, 0, st>>>(w, wm, wo, g, C, o); break;
        default: k_project_bwd_gather<TW, TG, 0><<<grid(w.N), TB, 0, st>>>(w, wm, wo, g, C, o); break;
    }
}

}  // namespace

int64_t transpose_scan_tiles(int64_t N) { return (N + TSCAN - 1) / TSCAN; }

int build_transpose(const WeightsView& w, int32_t* cnt, int32_t* ptr, int32_t* ent, int32_t* nodes, int32_t* tsum,
                    hipStream_t st) {
    const int64_t nt = transpose_scan_tiles(w.N);
    if (nt > (int64_t(1) << 30)) {
        set_error("too many particles for the particle-major index");
        return P2M_EINVAL;
    }
    int rc = fill_bytes_zero(cnt, sizeof(int32_t) * w.N, st);
    if (rc) return rc;
    const int64_t ne = entry_grid(w);
    k_tcount<<<grid(ne), TB, 0, st>>>(w, ne, cnt);
    k_tscan_tiles<<<static_cast<unsigned>(nt), TB, 0, st>>>(cnt, w.N, ptr, tsum);
    k_tscan_totals<<<1, TB, 0, st>>>(tsum, static_cast<int>(nt));
    k_tscan_add<<<grid(w.N + 1), TB, 0, st>>>(ptr, w.N, tsum, static_cast<int>(nt), cnt);
    k_tfill<<<grid(ne), TB, 0, st>>>(w, ne, ptr, cnt, ent, nodes);
    k_tsort<<<grid(w.N), TB, 0, st>>>(ptr, w.N, ent, nodes);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int project_backward_gather(const WeightsView& w, const void* grad_mesh, int C, int dtype, void* grad_vals,
                            hipStream_t st) {
    if (dtype == P2M_F64) launch_gather<double, double>(w, w.w64, w.ow64, grad_mesh, C, grad_vals, st);
    else launch_gather<float, float>(w, w.w32, w.ow32, grad_mesh, C, grad_vals, st);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int gather_entry_grads(const WeightsView& w, double* grad_pos, hipStream_t st) {
    k_gpos_gather<<<grid(w.N), TB, 0, st>>>(w, reinterpret_cast<double2*>(grad_pos));
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
