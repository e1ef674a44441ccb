// P2M weighted sum, eq. (p2m): mesh[i][c] = sum_mu psi_mu(r_i) vals[mu][c],
// and its adjoint for fixed weights.
//
// The ELL rows are stored per node slot (64 slots per 8 x 8 node tile, entry
// k of consecutive slots contiguous); a block takes one node tile and its
// quads walk the rows, gathering the C channels of each particle from the
// user-ordered value array.
#include "kernels.h"

namespace p2m {

namespace {


template <typename T> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };


// The mesh node of a quad's slot in a one-tile block (false beyond the mesh).
__device__ __forceinline__ bool tile_node(const WeightsView& wv, int64_t& slot, int64_t& node) {
    const int64_t tile = blockIdx.x;
    const SetDesc& sd = wv.sets[set_search(wv.S, tile, [&](int s) { return wv.sets[s].t0; })];
    slot = tile * TILE_N + (threadIdx.x >> 2);
    int i, j;
    if (!slot_ij(sd, slot, i, j)) return false;
    node = ij_node(sd, i, j);
    return true;
}

// vals element type TV, weights TW, output TO (accumulate in TW).  Four
// lanes per node: lane l takes ELL entries l, l + 4, ...; the partial sums
// are combined by a quad reduction (fixed order, so results are bitwise
// reproducible), and lane c % 4 stores channel c.
template <typename TV, typename TW, typename TO, int CC>
__device__ __forceinline__ void project_row(const WeightsView& wv, const TW* __restrict__ w,
                                            const TW* __restrict__ ow, const TV* __restrict__ vals, int C,
                                            int64_t slot, int64_t node, int lane, TO* __restrict__ out) {
    const int64_t ns = wv.n_slots;
    RowSum<TV, TW, TO, CC> rs;
    rs.init();
    const int cnt = row_len(wv.meta[slot]);
    const int ce = cnt < KMAX ? cnt : KMAX;
    for (int k = lane; k < ce; k += 4) rs.add(w[k * ns + slot], vals, wv.idx[k * ns + slot], C);
    if (cnt > KMAX) {
        // a long row's entries KMAX.. (overflow row)
        const int32_t r = wv.orow[slot];
        for (int k = KMAX + lane; k < cnt; k += 4) {
            const int64_t o = ovf_at(wv.n_ovf, r, k);
            rs.add(ow[o], vals, wv.oidx[o], C);
        }
    }
    rs.store(out, node, C, lane);
}

template <typename TV, typename TW, typename TO, int CC>
__global__ void __launch_bounds__(256) k_project(WeightsView wv, const TW* __restrict__ w, const TW* __restrict__ ow,
                                                 const TV* __restrict__ vals, int Crt, TO* __restrict__ out) {
    const int lane = threadIdx.x & 3;
    int64_t slot, node;
    if (!tile_node(wv, slot, node)) return;  // the four lanes of a node leave together
    project_row<TV, TW, TO, CC>(wv, w, ow, vals, CC > 0 ? CC : Crt, slot, node, lane, out);
}

// The rows of the exact and rank-revealing paths after a fused build (whose
// other rows were projected as they were weighted): the slow-path list, then
// the rank-revealing list (a row on both is projected twice, to the same
// bits).  A quad per listed row, the grid looping over the lists.
template <typename TV, typename TW, typename TO, int CC>
__global__ void __launch_bounds__(256) k_project_list(WeightsView wv, const int32_t* __restrict__ slow,
                                                      const TW* __restrict__ w, const TW* __restrict__ ow,
                                                      const TV* __restrict__ vals, int Crt, TO* __restrict__ out) {
    const int lane = threadIdx.x & 3;
    const int ns = static_cast<int>(wv.diag[D_SLOWCNT]), nr = static_cast<int>(wv.diag[D_RDCNT]);
    const int stride = static_cast<int>(gridDim.x) * 64;
    for (int li = static_cast<int>(blockIdx.x) * 64 + static_cast<int>(threadIdx.x >> 2); li < ns + nr;
         li += stride) {
        const int64_t slot = li < ns ? slow[li] : static_cast<int64_t>(static_cast<uint32_t>(wv.rd[li - ns]) & ~RD_SOLVED);
        const SetDesc& sd = wv.sets[set_search(wv.S, slot / TILE_N, [&](int s) { return wv.sets[s].t0; })];
        int i, j;
        if (!slot_ij(sd, slot, i, j)) continue;
        project_row<TV, TW, TO, CC>(wv, w, ow, vals, CC > 0 ? CC : Crt, slot, ij_node(sd, i, j), lane, out);
    }
}

template <typename TV, typename TW, typename TO>
void launch_project(const WeightsView& wv, const TW* w, const TW* ow, const void* vals, int C, void* out,
                    hipStream_t st) {
    const int blocks = static_cast<int>(wv.n_slots / TILE_N);  // one node tile (64 quads) per block
    const TV* v = static_cast<const TV*>(vals);
    TO* o = static_cast<TO*>(out);
    switch (C) {
        case 1: k_project<TV, TW, TO, 1><<<blocks, 256, 0, st>>>(wv, w, ow, v, C, o); break;
        case 2: k_project<TV, TW, TO, 2><<<blocks, 256, 0, st>>>(wv, w, ow, v, C, o); break;
        case 3: k_project<TV, TW, TO, 3><<<blocks, 256, 0, st>>>(wv, w, ow, v, C, o); break;
        case 4: k_project<TV, TW, TO, 4><<<blocks, 256, 0, st>>>(wv, w, ow, v, C, o); break;
        default: k_project<TV, TW, TO, 0><<<blocks, 256, 0, st>>>(wv, w, ow, v, C, o); break;
    }
}

template <typename TV, typename TW, typename TO>
void launch_project_list(const WeightsView& wv, const int32_t* slow, const TW* w, const TW* ow, const void* vals,
                         int C, void* out, hipStream_t st) {
    const TV* v = static_cast<const TV*>(vals);
    TO* o = static_cast<TO*>(out);
    if (C == 3) k_project_list<TV, TW, TO, 3><<<64, 256, 0, st>>>(wv, slow, w, ow, v, C, o);
    else k_project_list<TV, TW, TO, 0><<<64, 256, 0, st>>>(wv, slow, w, ow, v, C, o);
}

// grad_vals[j][c] += w * grad_mesh[i][c] (atomics) ; grad_w[k][i] = sum_c grad_mesh[i][c] vals[j][c]
// (grad_w in mesh-node order [KROW][n_nodes]; entries past the row are
// zero).  A quad per row slot, in the tiles' slot order as the forward
// projection takes them: lane l takes entries l, l + 4, ..., so that four
// times as many rows are walked at once; for a fixed channel count (CC > 0)
// an entry's loads are all issued before its sums.
template <typename TV, typename TW, typename TG, int CC>
__global__ void __launch_bounds__(256) k_project_bwd(WeightsView wv, const TW* __restrict__ w,
                                                     const TW* __restrict__ ow, const TG* __restrict__ gmesh, int Crt,
                                                     const TV* __restrict__ vals, TG* __restrict__ gvals,
                                                     double* __restrict__ gw) {
    constexpr int NC = CC > 0 ? CC : CMAX;
    const int C = CC > 0 ? CC : Crt;
    const int64_t slot = static_cast<int64_t>(blockIdx.x) * TILE_N + (threadIdx.x >> 2);
    const int lane = threadIdx.x & 3;
    if (slot >= wv.n_slots) return;
    const SetDesc& sd = wv.sets[set_search(wv.S, slot / TILE_N, [&](int s) { return wv.sets[s].t0; })];
    int i, j;
    if (!slot_ij(sd, slot, i, j)) return;
    const int64_t node = ij_node(sd, i, j);
    const int64_t ns = wv.n_slots, nn = wv.n_nodes;
    const int cnt = row_len(wv.meta[slot]);
    TG g[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < C) g[c] = gmesh[node * C + c];
    const int32_t r = cnt > KMAX ? wv.orow[slot] : 0;
    for (int k = lane; k < cnt; k += 4) {
        const bool main = k < KMAX;
        const int64_t at = main ? k * ns + slot : ovf_at(wv.n_ovf, r, k);
        const int64_t p = main ? wv.idx[at] : wv.oidx[at];
        if (gvals) {
            const TG wk = static_cast<TG>(main ? w[at] : ow[at]);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < C) atomicAdd(&gvals[p * C + c], wk * g[c]);
        }
        if (gw) {
            double v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < C) v[c] = static_cast<double>(ld(vals, p * C + c));
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < C) s += static_cast<double>(g[c]) * v[c];
            gw[k * nn + node] = s;
        }
    }
    if (gw)
        for (int k = cnt + lane; k < KROW; k += 4) gw[k * nn + node] = 0.0;
}

template <typename TV, typename TW, typename TG>
void launch_project_bwd(const WeightsView& wv, const TW* w, const TW* ow, const TG* gmesh, int C, const TV* vals,
                        TG* gvals, double* gw, hipStream_t st) {
    const int blocks = static_cast<int>(wv.n_slots / TILE_N);
    switch (C) {
        case 1: k_project_bwd<TV, TW, TG, 1><<<blocks, 256, 0, st>>>(wv, w, ow, gmesh, C, vals, gvals, gw); break;
        case 2: k_project_bwd<TV, TW, TG, 2><<<blocks, 256, 0, st>>>(wv, w, ow, gmesh, C, vals, gvals, gw); break;
        case 3: k_project_bwd<TV, TW, TG, 3><<<blocks, 256, 0, st>>>(wv, w, ow, gmesh, C, vals, gvals, gw); break;
        case 4: k_project_bwd<TV, TW, TG, 4><<<blocks, 256, 0, st>>>(wv, w, ow, gmesh, C, vals, gvals, gw); break;
        default: k_project_bwd<TV, TW, TG, 0><<<blocks, 256, 0, st>>>(wv, w, ow, gmesh, C, vals, gvals, gw); break;
    }
}

}  // namespace

int project(const WeightsView& wv, const void* vals, int C, int dtype, void* mesh_vals, hipStream_t st) {
    PhaseTimer _timer(PH_PROJECT, st);
    if (dtype == P2M_F64) {
        launch_project<double, double, double>(wv, wv.w64, wv.ow64, vals, C, mesh_vals, st);
    } else {
        if (!wv.w32) {
            set_error("p2m_project: FP32/BF16 values need a handle built with P2M_WEIGHTS_F32");
            return P2M_EINVAL;
        }
        if (dtype == P2M_F32)
            launch_project<float, float, float>(wv, wv.w32, wv.ow32, vals, C, mesh_vals, st);
        else
            launch_project<uint16_t, float, float>(wv, wv.w32, wv.ow32, vals, C, mesh_vals, st);
    }
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int project_listed(const WeightsView& wv, const int32_t* slow, const void* vals, int C, int dtype, void* mesh_vals,
                   hipStream_t st) {
    if (dtype == P2M_F64) launch_project_list<double, double, double>(wv, slow, wv.w64, wv.ow64, vals, C, mesh_vals, st);
    else if (dtype == P2M_F32) launch_project_list<float, float, float>(wv, slow, wv.w32, wv.ow32, vals, C, mesh_vals, st);
    else launch_project_list<uint16_t, float, float>(wv, slow, wv.w32, wv.ow32, vals, C, mesh_vals, st);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int project_backward(const WeightsView& wv, const void* grad_mesh, int C, int dtype, const void* vals,
                     void* grad_vals, double* grad_w, hipStream_t st) {
    PhaseTimer _timer(PH_PROJECT_BWD, st);
    if (dtype != P2M_F64 && !wv.w32) {
        set_error("p2m_project_backward: FP32/BF16 needs a handle built with P2M_WEIGHTS_F32");
        return P2M_EINVAL;
    }
    if (grad_vals && wv.tptr) {
        // a particle-major index: grad_vals gathered per particle (no
        // atomics); the row pass below then forms grad_w alone
        int rc = project_backward_gather(wv, grad_mesh, C, dtype, grad_vals, st);
        if (rc) return rc;
        grad_vals = nullptr;
        if (!grad_w) return P2M_OK;
    }
    if (dtype == P2M_F64) {
        if (grad_vals) {
            int rc = fill_bytes_zero(grad_vals, sizeof(double) * wv.N * C, st);
            if (rc) return rc;
        }
        launch_project_bwd<double, double, double>(wv, wv.w64, wv.ow64, static_cast<const double*>(grad_mesh), C,
                                                   static_cast<const double*>(vals),
                                                   static_cast<double*>(grad_vals), grad_w, st);
    } else {
        if (grad_vals) {
            int rc = fill_bytes_zero(grad_vals, sizeof(float) * wv.N * C, st);
            if (rc) return rc;
        }
        if (dtype == P2M_F32)
            launch_project_bwd<float, float, float>(wv, wv.w32, wv.ow32, static_cast<const float*>(grad_mesh), C,
                                                    static_cast<const float*>(vals),
                                                    static_cast<float*>(grad_vals), grad_w, st);
        else
            launch_project_bwd<uint16_t, float, float>(wv, wv.w32, wv.ow32, static_cast<const float*>(grad_mesh), C,
                                                       static_cast<const uint16_t*>(vals),
                                                       static_cast<float*>(grad_vals), grad_w, st);
    }
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
