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

// Slot of node `node` (handle numbering) and its row length.
__device__ __forceinline__ int64_t node_row(const WeightsView& w, int64_t node, int& n, int32_t& orow) {
    const SetDesc& sd = w.sets[set_search(w.S, node, [&](int s) { return w.sets[s].n0; })];
    const int64_t ln = node - sd.n0;
    const int64_t slot = node_slot(sd, static_cast<int>(ln % (sd.m.nx + 1)), static_cast<int>(ln / (sd.m.nx + 1)));
    n = row_len(w.meta[slot]);
    orow = n > KMAX ? w.orow[slot] : 0;
    return slot;
}

// User id of entry k of a row.
__device__ __forceinline__ int32_t entry_uid(const WeightsView& w, int64_t slot, int32_t orow, int k) {
    return k < KMAX ? w.idx[k * w.n_slots + slot] : w.oidx[ovf_at(w.n_ovf, orow, k)];
}

// 1. entries per particle
__global__ void __launch_bounds__(TB) k_tcount(WeightsView w, int32_t* __restrict__ cnt) {
    const int64_t node = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (node >= w.n_nodes) return;
    int n;
    int32_t orow;
    const int64_t slot = node_row(w, node, n, orow);
    for (int k = 0; k < n; ++k) atomicAdd(&cnt[entry_uid(w, slot, orow, k)], 1);
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
__global__ void __launch_bounds__(TB) k_tfill(WeightsView w, const int32_t* __restrict__ ptr,
                                             int32_t* __restrict__ cur, int32_t* __restrict__ ent,
                                             int32_t* __restrict__ nodes) {
    const int64_t node = static_cast<int64_t>(blockIdx.x) * TB + threadIdx.x;
    if (node >= w.n_nodes) return;
    int n;
    int32_t orow;
    const int64_t slot = node_row(w, node, n, orow);
    for (int k = 0; k < n; ++k) {
        const int32_t u = entry_uid(w, slot, orow, k);
        const int32_t at = ptr[u] + atomicAdd(&cur[u], 1);
        ent[at] = static_cast<int32_t>(entry_at(w.n_slots, w.n_ovf, orow, slot, k));
        nodes[at] = static_cast<int32_t>(node);
    }
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
    k_tcount<<<grid(w.n_nodes), TB, 0, st>>>(w, cnt);
    k_tscan_tiles<<<static_cast<unsigned>(nt), TB, 0, st>>>(cnt, w.N, ptr, tsum);
    k_tscan_totals<<<1, TB, 0, st>>>(tsum, static_cast<int>(nt));
    k_tscan_add<<<grid(w.N + 1), TB, 0, st>>>(ptr, w.N, tsum, static_cast<int>(nt), cnt);
    k_tfill<<<grid(w.n_nodes), TB, 0, st>>>(w, ptr, cnt, ent, nodes);
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
