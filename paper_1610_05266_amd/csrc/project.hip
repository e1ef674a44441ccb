// P2M weighted sum, eq. (p2m): mesh[i][c] = sum_mu psi_mu(r_i) vals[mu][c],
// and its adjoint for fixed weights.
//
// One thread per mesh node walks its ELL row (slot-major layout, so the k-th
// entries of consecutive nodes are contiguous) and gathers the C channels of
// each particle from the user-ordered value array.
#include "kernels.h"

namespace p2m {

namespace {

constexpr int CMAX = 16;

template <typename T> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };

__device__ __forceinline__ double ld(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ld(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ld(const uint16_t* p, int64_t i) { return bf16_to_f32(p[i]); }

// vals element type TV, weights TW, output TO (accumulate in TW).  Four
// lanes per node: lane l takes ELL entries l, l + 4, ...; the partial sums
// are combined by a quad reduction (fixed order, so results are bitwise
// reproducible), and lane c % 4 stores channel c.
template <typename TV, typename TW, typename TO, int CC>
__global__ void __launch_bounds__(256) k_project(const uint32_t* __restrict__ meta, const int32_t* __restrict__ idx,
                                                 const TW* __restrict__ w, int64_t n_nodes,
                                                 const TV* __restrict__ vals, int Crt, TO* __restrict__ out) {
    constexpr int NC = CC > 0 ? CC : CMAX;
    const int lane = threadIdx.x & 3;
    const int64_t node = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 2;
    if (node >= n_nodes) return;  // the four lanes of a node leave together
    const int C = CC > 0 ? CC : Crt;
    TW acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = TW(0);
    const int cnt = row_len(meta[node]);
    for (int k = lane; k < cnt; k += 4) {
        const int64_t j = idx[k * n_nodes + node];
        const TW wk = w[k * n_nodes + node];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < C) acc[c] += wk * static_cast<TW>(ld(vals, j * C + c));
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c >= C) break;
        TW v = acc[c];
        v += lane_xor<4>(v, 1);
        v += lane_xor<4>(v, 2);
        if (lane == (c & 3)) out[node * C + c] = static_cast<TO>(v);
    }
}

template <typename TV, typename TW, typename TO>
void launch_project(const WeightsView& wv, const TW* w, const void* vals, int C, void* out, hipStream_t st) {
    const int blocks = static_cast<int>((4 * wv.n_nodes + 255) / 256);
    const TV* v = static_cast<const TV*>(vals);
    TO* o = static_cast<TO*>(out);
    switch (C) {
        case 1: k_project<TV, TW, TO, 1><<<blocks, 256, 0, st>>>(wv.meta, wv.idx, w, wv.n_nodes, v, C, o); break;
        case 2: k_project<TV, TW, TO, 2><<<blocks, 256, 0, st>>>(wv.meta, wv.idx, w, wv.n_nodes, v, C, o); break;
        case 3: k_project<TV, TW, TO, 3><<<blocks, 256, 0, st>>>(wv.meta, wv.idx, w, wv.n_nodes, v, C, o); break;
        case 4: k_project<TV, TW, TO, 4><<<blocks, 256, 0, st>>>(wv.meta, wv.idx, w, wv.n_nodes, v, C, o); break;
        default: k_project<TV, TW, TO, 0><<<blocks, 256, 0, st>>>(wv.meta, wv.idx, w, wv.n_nodes, v, C, o); break;
    }
}

// grad_vals[j][c] += w * grad_mesh[i][c] (atomics) ; grad_w[k][i] = sum_c grad_mesh[i][c] vals[j][c]
template <typename TV, typename TW, typename TG>
__global__ void __launch_bounds__(256) k_project_bwd(const uint32_t* __restrict__ meta,
                                                     const int32_t* __restrict__ idx, const TW* __restrict__ w,
                                                     int64_t n_nodes, const TG* __restrict__ gmesh, int C,
                                                     const TV* __restrict__ vals, TG* __restrict__ gvals,
                                                     double* __restrict__ gw) {
    const int64_t node = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (node >= n_nodes) return;
    const int cnt = row_len(meta[node]);
    TG g[CMAX];
    for (int c = 0; c < C; ++c) g[c] = gmesh[node * C + c];
    for (int k = 0; k < cnt; ++k) {
        const int64_t j = idx[k * n_nodes + node];
        if (gvals) {
            const TG wk = static_cast<TG>(w[k * n_nodes + node]);
            for (int c = 0; c < C; ++c) atomicAdd(&gvals[j * C + c], wk * g[c]);
        }
        if (gw) {
            double s = 0.0;
            for (int c = 0; c < C; ++c) s += static_cast<double>(g[c]) * static_cast<double>(ld(vals, j * C + c));
            gw[k * n_nodes + node] = s;
        }
    }
    if (gw)
        for (int k = cnt; k < KMAX; ++k) gw[k * n_nodes + node] = 0.0;
}

}  // namespace

int project(const WeightsView& wv, const void* vals, int C, int dtype, void* mesh_vals, hipStream_t st) {
    PhaseTimer _timer(PH_PROJECT, st);
    if (dtype == P2M_F64) {
        launch_project<double, double, double>(wv, wv.w64, vals, C, mesh_vals, st);
    } else {
        if (!wv.w32) {
            set_error("p2m_project: FP32/BF16 values need a handle built with P2M_WEIGHTS_F32");
            return P2M_EINVAL;
        }
        if (dtype == P2M_F32)
            launch_project<float, float, float>(wv, wv.w32, vals, C, mesh_vals, st);
        else
            launch_project<uint16_t, float, float>(wv, wv.w32, vals, C, mesh_vals, st);
    }
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int project_backward(const WeightsView& wv, const void* grad_mesh, int C, int dtype, const void* vals,
                     void* grad_vals, double* grad_w, hipStream_t st) {
    PhaseTimer _timer(PH_PROJECT_BWD, st);
    const int blocks = static_cast<int>((wv.n_nodes + 255) / 256);
    if (dtype == P2M_F64) {
        if (grad_vals) {
            int rc = fill_bytes_zero(grad_vals, sizeof(double) * wv.N * C, st);
            if (rc) return rc;
        }
        k_project_bwd<double, double, double><<<blocks, 256, 0, st>>>(
            wv.meta, wv.idx, wv.w64, wv.n_nodes, static_cast<const double*>(grad_mesh), C,
            static_cast<const double*>(vals), static_cast<double*>(grad_vals), grad_w);
    } else {
        if (!wv.w32) {
            set_error("p2m_project_backward: FP32/BF16 needs a handle built with P2M_WEIGHTS_F32");
            return P2M_EINVAL;
        }
        if (grad_vals) {
            int rc = fill_bytes_zero(grad_vals, sizeof(float) * wv.N * C, st);
            if (rc) return rc;
        }
        if (dtype == P2M_F32)
            k_project_bwd<float, float, float><<<blocks, 256, 0, st>>>(
                wv.meta, wv.idx, wv.w32, wv.n_nodes, static_cast<const float*>(grad_mesh), C,
                static_cast<const float*>(vals), static_cast<float*>(grad_vals), grad_w);
        else
            k_project_bwd<uint16_t, float, float><<<blocks, 256, 0, st>>>(
                wv.meta, wv.idx, wv.w32, wv.n_nodes, static_cast<const float*>(grad_mesh), C,
                static_cast<const uint16_t*>(vals), static_cast<float*>(grad_vals), grad_w);
    }
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
