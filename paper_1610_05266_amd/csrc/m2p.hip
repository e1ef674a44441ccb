// M2P, eq. (m2p), with the fixed mesh's linear FE shape functions, and its
// adjoint.
//
// The mesh is uniform, so locating a particle is arithmetic: cell
// i = min(floor((x - x0)/H), nx - 1) (same in y), local coordinates
// xi = (x - x0)/H - i, eta likewise; the cell's diagonal (i,j)-(i+1,j+1)
// splits it into the triangle with xi >= eta (nodes (i,j), (i+1,j), (i+1,j+1),
// weights 1-xi, xi-eta, eta) and the one with xi < eta (nodes (i,j),
// (i+1,j+1), (i,j+1), weights 1-eta, xi, eta-xi).  One thread per particle:
// 16 bytes of position in, C values out, three gathers from the mesh array
// (small enough to stay in the last-level cache).
#include "kernels.h"

namespace p2m {

namespace {


struct Loc {
    int64_t n0, n1, n2;
    double w0, w1, w2;
    bool lower, ok;
};

// The particle's cell and local coordinates (the first half of locating
// it), and the triangle's nodes and weights from them (the second half):
// split so that a kernel can keep the first and finish later with the same
// bits.
struct Cell {
    int64_t n00;  // the cell's lower-left node (index within the set)
    double xi, eta;
    bool lower, ok;
};

__device__ __forceinline__ Cell cell_of(const MeshD& m, double2 p) {
    Cell c;
    const double x1 = add_rn(m.x0, mul_rn(static_cast<double>(m.nx), m.H));
    const double y1 = add_rn(m.y0, mul_rn(static_cast<double>(m.ny), m.H));
    c.ok = p.x >= m.x0 && p.x <= x1 && p.y >= m.y0 && p.y <= y1;
    const double tx = (p.x - m.x0) / m.H;
    const double ty = (p.y - m.y0) / m.H;
    // clamp in floating point first (NaN and huge values included)
    const int i = static_cast<int>(fmax(fmin(floor(tx), static_cast<double>(m.nx - 1)), 0.0));
    const int j = static_cast<int>(fmax(fmin(floor(ty), static_cast<double>(m.ny - 1)), 0.0));
    c.xi = tx - i;
    c.eta = ty - j;
    c.n00 = static_cast<int64_t>(j) * (m.nx + 1) + i;
    c.lower = c.xi >= c.eta;
    return c;
}

__device__ __forceinline__ Loc loc_of(const MeshD& m, const Cell& c) {
    Loc L;
    const int64_t s = m.nx + 1;
    L.ok = c.ok;
    L.lower = c.lower;
    L.n0 = c.n00;
    if (c.lower) {
        L.n1 = c.n00 + 1;
        L.n2 = c.n00 + s + 1;
        L.w0 = 1.0 - c.xi;
        L.w1 = c.xi - c.eta;
        L.w2 = c.eta;
    } else {
        L.n1 = c.n00 + s + 1;
        L.n2 = c.n00 + s;
        L.w0 = 1.0 - c.eta;
        L.w1 = c.xi;
        L.w2 = c.eta - c.xi;
    }
    return L;
}

__device__ __forceinline__ Loc locate_cell(const MeshD& m, double2 p) { return loc_of(m, cell_of(m, p)); }

__device__ __forceinline__ double ldm(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldm(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ void st(double* p, int64_t i, double v) { p[i] = v; }
__device__ __forceinline__ void st(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void st(uint16_t* p, int64_t i, float v) { p[i] = f32_to_bf16(v); }
__device__ __forceinline__ double ldv(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const float* p, int64_t i) { return p[i]; }

// The mesh of particle mu and the offset of that mesh's nodes: one mesh, or
// the set of a batch that holds mu.
struct MeshOf {
    MeshD m;
    const SetDesc* sets;
    int S;
    __device__ __forceinline__ MeshD get(int64_t mu, int64_t& n0) const {
        if (!sets) {
            n0 = 0;
            return m;
        }
        const SetDesc& sd = sets[set_search(S, mu, [&](int s) { return sets[s].p0; })];
        n0 = sd.n0;
        return sd.m;
    }
};

// TM mesh value type, TO particle output type.  The three products are
// summed in FP64 and rounded once: with FP32 storage the output is the
// correctly rounded value of the interpolant (BF16: rounded through FP32),
// not a sum of rounded products (a position gradient taken through these
// values amplifies their rounding by |a| / (h |grad a|), some hundreds on
// fine meshes, so an extra rounding of a sum would show).
// PPT particles per thread, strided by the block size (coalesced): all their
// position loads are issued before the first is used, then all their cells
// are located and all their mesh gathers issued before the first sum, so
// that a wave keeps every load of its particles in flight at once.
template <typename TM, typename TO, int CC, int PPT>
__global__ void __launch_bounds__(256) k_m2p(MeshOf mo, const TM* __restrict__ mv, int Crt,
                                             const double2* __restrict__ pos, int64_t N, TO* __restrict__ out) {
    constexpr int NC = CC > 0 ? CC : CMAX;
    const int C = CC > 0 ? CC : Crt;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (256 * PPT) + threadIdx.x;
    double2 p[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t mu = base + k * 256;
        p[k] = pos[mu < N ? mu : N - 1];
    }
    // per particle only what the sums need: the three weights and the
    // element offsets of the three nodes (32-bit: the host keeps C times the
    // node count below 2^31), NaN weights marking a particle off its mesh
    double w[PPT][3];
    int32_t o[PPT][3];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t mu = base + k * 256;
        int64_t n0;
        const MeshD m = mo.get(mu < N ? mu : N - 1, n0);
        const Loc L = locate_cell(m, p[k]);
        w[k][0] = L.ok ? L.w0 : NAN;
        w[k][1] = L.w1;
        w[k][2] = L.w2;
        o[k][0] = static_cast<int32_t>((L.n0 + n0) * C);
        o[k][1] = static_cast<int32_t>((L.n1 + n0) * C);
        o[k][2] = static_cast<int32_t>((L.n2 + n0) * C);
    }
    TM g[PPT][3][NC];
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < C)
#pragma unroll
                for (int t = 0; t < 3; ++t) g[k][t][c] = ldm(mv, o[k][t] + c);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t mu = base + k * 256;
        if (mu >= N) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < C) {
                const double v = w[k][0] * static_cast<double>(g[k][0][c]) + w[k][1] * static_cast<double>(g[k][1][c]) +
                                 w[k][2] * static_cast<double>(g[k][2][c]);
                st(out, mu * C + c, static_cast<TM>(v));
            }
    }
}

template <typename TM, typename TO, int PPT>
void launch_m2p_ppt(const MeshOf& m, const TM* M, int C, const double2* P, int64_t N, TO* O, hipStream_t s) {
    const int blocks = static_cast<int>((N + 256 * PPT - 1) / (256 * PPT));
    switch (C) {
        case 1: k_m2p<TM, TO, 1, PPT><<<blocks, 256, 0, s>>>(m, M, C, P, N, O); break;
        case 2: k_m2p<TM, TO, 2, PPT><<<blocks, 256, 0, s>>>(m, M, C, P, N, O); break;
        case 3: k_m2p<TM, TO, 3, PPT><<<blocks, 256, 0, s>>>(m, M, C, P, N, O); break;
        default: k_m2p<TM, TO, 4, PPT><<<blocks, 256, 0, s>>>(m, M, C, P, N, O); break;
    }
}

// ppt: particles per thread (1, 2 or 4; a performance option, the results
// do not depend on it).  More than four channels: one particle per thread,
// the gathered values of up to CMAX channels in registers.
template <typename TM, typename TO>
void launch_m2p(const MeshOf& m, const void* mv, int C, const double* pos, int64_t N, void* out, int ppt,
                hipStream_t s) {
    const TM* M = static_cast<const TM*>(mv);
    const double2* P = reinterpret_cast<const double2*>(pos);
    TO* O = static_cast<TO*>(out);
    if (C > 4) {
        k_m2p<TM, TO, 0, 1><<<static_cast<int>((N + 255) / 256), 256, 0, s>>>(m, M, C, P, N, O);
        return;
    }
    if (ppt >= 4) launch_m2p_ppt<TM, TO, 4>(m, M, C, P, N, O, s);
    else if (ppt == 2) launch_m2p_ppt<TM, TO, 2>(m, M, C, P, N, O, s);
    else launch_m2p_ppt<TM, TO, 1>(m, M, C, P, N, O, s);
}

// Offsets (relative to an edge's first end) of the ten support slots of a
// horizontal, vertical and diagonal edge, in the order of the edge table's
// rows.
constexpr int kSupOff[3][10][2] = {
    {{-1, -1}, {-1, 0}, {0, -1}, {0, 0}, {0, 1}, {1, -1}, {1, 0}, {1, 1}, {2, 0}, {2, 1}},
    {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 0}, {0, 1}, {0, 2}, {1, 0}, {1, 1}, {1, 2}},
    {{-1, -1}, {-1, 0}, {0, -1}, {0, 0}, {0, 1}, {1, 0}, {1, 1}, {1, 2}, {2, 1}, {2, 2}}};

// M2P with the mesh's quadratically consistent functions (App. B on the
// mesh): the linear part above plus, for each edge (p, q) of the particle's
// triangle, 2 phi_p phi_q times the edge's stencil of ten coefficients
// (table row, computed once per mesh).  The triangle's edges in the order
// (0,1), (1,2), (0,2): lower triangle horizontal (i,j), vertical (i+1,j),
// diagonal (i,j); upper triangle diagonal (i,j), horizontal (i,j+1),
// vertical (i,j).  One thread per particle.
template <typename TM, typename TO, int CC, bool PER>
__global__ void __launch_bounds__(256) k_m2p_qcsf(MeshD m, const int32_t* __restrict__ eidx,
                                                  const double* __restrict__ ecoef, const TM* __restrict__ mv,
                                                  int Crt, const double2* __restrict__ pos, int64_t N,
                                                  TO* __restrict__ out) {
    constexpr bool per = PER;
    constexpr int NC = CC > 0 ? CC : CMAX;
    const int64_t mu = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (mu >= N) return;
    const int C = CC > 0 ? CC : Crt;
    const Loc L = locate_cell(m, pos[mu]);
    const int64_t s = m.nx + 1;
    const int i = static_cast<int>(L.n0 % s), j = static_cast<int>(L.n0 / s);
    const int64_t nh = static_cast<int64_t>(m.nx) * (m.ny + 1), nv = s * m.ny;
    const int64_t eh = static_cast<int64_t>(j) * m.nx + i, ed = nh + nv + static_cast<int64_t>(j) * m.nx + i;
    const int64_t e01 = L.lower ? eh : ed;
    const int64_t e12 = L.lower ? nh + static_cast<int64_t>(j) * s + i + 1 : eh + m.nx;
    const int64_t e02 = L.lower ? ed : nh + static_cast<int64_t>(j) * s + i;
    const double c01 = 2.0 * L.w0 * L.w1, c12 = 2.0 * L.w1 * L.w2, c02 = 2.0 * L.w0 * L.w2;
    // A cell at least one cell from the wall has complete supports on all
    // three edges, whose coefficients then equal those of the same
    // orientation at node (1, 1) (the construction is translation
    // invariant): every such particle reads those three rows (the same
    // addresses for all, cached) and shifts their node ids, instead of three
    // rows of its own.
    // In a periodic box every edge is such an edge, and the node ids wrap
    // across the box sides (to the first column and row, which the last
    // repeat).
    const bool inner = per || (m.nx >= 3 && m.ny >= 3 && i >= 1 && j >= 1 && i + 2 <= m.nx && j + 2 <= m.ny);
    const int64_t r11 = s + 1, rh = m.nx + 1, rv = nh + s + 1, rd = nh + nv + m.nx + 1;
    const int64_t n00 = L.n0;
    TM acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = TM(0);
    if (inner) {
        // the node weights on the 4 x 4 offsets (-1..2)^2 from node (i, j):
        // linear part, then each edge's stencil at its place (lower: H at
        // (0,0), V at (1,0), D at (0,0); upper: D at (0,0), H at (0,1), V at
        // (0,0)), both triangles' placements written with the other's
        // coefficients zero so that every index is a constant; then one
        // gather per node (14 offsets can carry weight) instead of one per
        // stencil entry
        double g[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) g[k] = 0.0;
        g[5] += L.w0;                       // (0,0)
        g[6] += L.lower ? L.w1 : 0.0;       // (1,0)
        g[10] += L.lower ? L.w2 : L.w1;     // (1,1)
        g[9] += L.lower ? 0.0 : L.w2;       // (0,1)
        const double cH0 = L.lower ? c01 : 0.0, cH1 = L.lower ? 0.0 : c12;
        const double cV1 = L.lower ? c12 : 0.0, cV0 = L.lower ? 0.0 : c02;
        const double cD = L.lower ? c02 : c01;
        const double* rowH = ecoef + rh * MESH_SUP;
        const double* rowV = ecoef + rv * MESH_SUP;
        const double* rowD = ecoef + rd * MESH_SUP;
#pragma unroll
        for (int k = 0; k < MESH_SUP; ++k) {
            const double aH = rowH[k], aV = rowV[k], aD = rowD[k];
            g[(kSupOff[0][k][1] + 1) * 4 + kSupOff[0][k][0] + 1] += cH0 * aH;
            g[(kSupOff[0][k][1] + 2) * 4 + kSupOff[0][k][0] + 1] += cH1 * aH;
            g[(kSupOff[1][k][1] + 1) * 4 + kSupOff[1][k][0] + 2] += cV1 * aV;
            g[(kSupOff[1][k][1] + 1) * 4 + kSupOff[1][k][0] + 1] += cV0 * aV;
            g[(kSupOff[2][k][1] + 1) * 4 + kSupOff[2][k][0] + 1] += cD * aD;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k == 3 || k == 12) continue;  // offsets (2,-1) and (-1,2): never in a support
            int64_t node = n00 + static_cast<int64_t>(k / 4 - 1) * s + (k % 4 - 1);
            if (per) {
                int a = i + (k % 4 - 1), b = j + (k / 4 - 1);
                a += a < 0 ? m.nx : (a >= m.nx ? -m.nx : 0);
                b += b < 0 ? m.ny : (b >= m.ny ? -m.ny : 0);
                node = static_cast<int64_t>(b) * s + a;
            }
            const TM f = static_cast<TM>(g[k]);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < C) acc[c] += f * ldm(mv, node * C + c);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < C) st(out, mu * C + c, L.ok ? acc[c] : static_cast<TM>(NAN));
        return;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < C)
            acc[c] = static_cast<TM>(L.w0) * ldm(mv, L.n0 * C + c) + static_cast<TM>(L.w1) * ldm(mv, L.n1 * C + c) +
                     static_cast<TM>(L.w2) * ldm(mv, L.n2 * C + c);
    // edge e (first end node a) or, inside, its representative r
    auto edge = [&](int64_t e, int64_t r, int64_t a, double ce) {
        const int64_t row = inner ? r : e, shift = inner ? a - r11 : 0;
#pragma unroll
        for (int k = 0; k < MESH_SUP; ++k) {
            const int64_t node = eidx[row * MESH_SUP + k] + shift;
            const TM f = static_cast<TM>(ce * ecoef[row * MESH_SUP + k]);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < C) acc[c] += f * ldm(mv, node * C + c);
        }
    };
    // lower: horizontal (i,j), vertical (i+1,j), diagonal (i,j);
    // upper: diagonal (i,j), horizontal (i,j+1), vertical (i,j)
    edge(e01, L.lower ? rh : rd, n00, c01);
    edge(e12, L.lower ? rv : rh, L.lower ? n00 + 1 : n00 + s, c12);
    edge(e02, L.lower ? rd : rv, n00, c02);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < C) st(out, mu * C + c, L.ok ? acc[c] : static_cast<TM>(NAN));
}

template <typename TM, typename TO, bool PER>
void launch_m2p_qcsf(const MeshD& m, const int32_t* idx, const double* coef, const void* mv, int C,
                     const double* pos, int64_t N, void* out, hipStream_t s) {
    const int blocks = static_cast<int>((N + 255) / 256);
    const TM* M = static_cast<const TM*>(mv);
    const double2* P = reinterpret_cast<const double2*>(pos);
    TO* O = static_cast<TO*>(out);
    switch (C) {
        case 1: k_m2p_qcsf<TM, TO, 1, PER><<<blocks, 256, 0, s>>>(m, idx, coef, M, C, P, N, O); break;
        case 2: k_m2p_qcsf<TM, TO, 2, PER><<<blocks, 256, 0, s>>>(m, idx, coef, M, C, P, N, O); break;
        case 3: k_m2p_qcsf<TM, TO, 3, PER><<<blocks, 256, 0, s>>>(m, idx, coef, M, C, P, N, O); break;
        case 4: k_m2p_qcsf<TM, TO, 4, PER><<<blocks, 256, 0, s>>>(m, idx, coef, M, C, P, N, O); break;
        default: k_m2p_qcsf<TM, TO, 0, PER><<<blocks, 256, 0, s>>>(m, idx, coef, M, C, P, N, O); break;
    }
}

// grad_mesh += phi_i(r_mu) g_mu (atomics); grad_pos[mu] += sum_c g_mu,c grad u_c.
// For a fixed channel count (CC > 0) every load of the particle (its
// upstream gradient and the nine mesh values) is issued before the first
// sum, as in the forward kernel.
template <typename TM, int CC>
__global__ void __launch_bounds__(256) k_m2p_bwd(MeshOf mo, const TM* __restrict__ mv, int Crt,
                                                 const double2* __restrict__ pos, int64_t N,
                                                 const TM* __restrict__ gv, TM* __restrict__ gmesh,
                                                 double2* __restrict__ gpos) {
    constexpr int NC = CC > 0 ? CC : 1;
    const int C = CC > 0 ? CC : Crt;
    const int64_t mu = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (mu >= N) return;
    int64_t n0;
    const MeshD m = mo.get(mu, n0);
    Loc L = locate_cell(m, pos[mu]);
    if (!L.ok) return;
    L.n0 += n0;
    L.n1 += n0;
    L.n2 += n0;
    // d(weights)/dxi and d/deta on the particle's triangle
    const double dxi0 = L.lower ? -1.0 : 0.0, dxi1 = 1.0, dxi2 = L.lower ? 0.0 : -1.0;
    const double det0 = L.lower ? 0.0 : -1.0, det1 = L.lower ? -1.0 : 0.0, det2 = 1.0;
    double gx = 0.0, gy = 0.0;
    if constexpr (CC > 0) {
        TM g[NC], v[3][NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) g[c] = gv[mu * C + c];
        if (gpos) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                v[0][c] = mv[L.n0 * C + c];
                v[1][c] = mv[L.n1 * C + c];
                v[2][c] = mv[L.n2 * C + c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (gmesh) {
                atomicAdd(&gmesh[L.n0 * C + c], static_cast<TM>(L.w0) * g[c]);
                atomicAdd(&gmesh[L.n1 * C + c], static_cast<TM>(L.w1) * g[c]);
                atomicAdd(&gmesh[L.n2 * C + c], static_cast<TM>(L.w2) * g[c]);
            }
            if (gpos) {
                const double v0 = v[0][c], v1 = v[1][c], v2 = v[2][c];
                const double gd = static_cast<double>(g[c]);
                gx += gd * (dxi0 * v0 + dxi1 * v1 + dxi2 * v2);
                gy += gd * (det0 * v0 + det1 * v1 + det2 * v2);
            }
        }
    } else {
        for (int c = 0; c < C; ++c) {
            const TM g = gv[mu * C + c];
            if (gmesh) {
                atomicAdd(&gmesh[L.n0 * C + c], static_cast<TM>(L.w0) * g);
                atomicAdd(&gmesh[L.n1 * C + c], static_cast<TM>(L.w1) * g);
                atomicAdd(&gmesh[L.n2 * C + c], static_cast<TM>(L.w2) * g);
            }
            if (gpos) {
                const double v0 = ldm(mv, L.n0 * C + c), v1 = ldm(mv, L.n1 * C + c), v2 = ldm(mv, L.n2 * C + c);
                const double gd = static_cast<double>(g);
                gx += gd * (dxi0 * v0 + dxi1 * v1 + dxi2 * v2);
                gy += gd * (det0 * v0 + det1 * v1 + det2 * v2);
            }
        }
    }
    if (gpos) {
        double2 a = gpos[mu];
        a.x += gx / m.H;
        a.y += gy / m.H;
        gpos[mu] = a;
    }
}

template <typename TM>
void launch_m2p_bwd(const MeshOf& m, const TM* mv, int C, const double2* P, int64_t N, const TM* gv, TM* gmesh,
                    double2* gpos, hipStream_t st) {
    const int blocks = static_cast<int>((N + 255) / 256);
    switch (C) {
        case 1: k_m2p_bwd<TM, 1><<<blocks, 256, 0, st>>>(m, mv, C, P, N, gv, gmesh, gpos); break;
        case 2: k_m2p_bwd<TM, 2><<<blocks, 256, 0, st>>>(m, mv, C, P, N, gv, gmesh, gpos); break;
        case 3: k_m2p_bwd<TM, 3><<<blocks, 256, 0, st>>>(m, mv, C, P, N, gv, gmesh, gpos); break;
        case 4: k_m2p_bwd<TM, 4><<<blocks, 256, 0, st>>>(m, mv, C, P, N, gv, gmesh, gpos); break;
        default: k_m2p_bwd<TM, 0><<<blocks, 256, 0, st>>>(m, mv, C, P, N, gv, gmesh, gpos); break;
    }
}

// grad_mesh of M2P as a gather: a quad per mesh node, nodes in the 8 x 8
// tiles of a weights handle built from the same positions.  The node takes
// every particle of the bins around its (up to four) cells, with one bin of
// margin (a particle's bin and its cell can differ by rounding on a cell
// side), locates it exactly as the forward does and adds its weight for
// this node: the sum over the particles whose triangle holds the node, with
// no atomics, in a fixed order (deterministic).  Lane l takes the particles
// l, l + 4, ... of each bin row of the node's window; FP64 sums, one
// rounding.
//
// The windows of a tile's nodes overlap (each particle lies in the windows
// of about nine nodes), so the block first locates every particle of the
// union of its nodes' windows once, into LDS (cell, local coordinates, user
// id), and the nodes then read those; a union too large for the LDS arrays
// (dense clusters, very fine bins) makes the block locate per node instead.
// Both ways visit the same particles in the same order with the same
// arithmetic: the sums are equal bit for bit.
constexpr int MB_ROWS = 64;    // bin rows of a tile's window held in LDS
constexpr int MB_CAP = 1920;   // particles of a tile's window held in LDS
constexpr int MB_PT = (MB_CAP + 255) / 256;  // of them per thread
constexpr int MB_WAVE = 64;

template <typename TG, int CC>
__global__ void __launch_bounds__(256) k_m2p_bwd_gather(WeightsView wv, const TG* __restrict__ gv, int Crt,
                                                        TG* __restrict__ gmesh) {
    constexpr int NC = CC > 0 ? CC : CMAX;
    const int C = CC > 0 ? CC : Crt;
    __shared__ double s_xi[MB_CAP], s_eta[MB_CAP];
    __shared__ int32_t s_code[MB_CAP], s_uid[MB_CAP];
    __shared__ int32_t s_off[MB_ROWS + 1];
    // start of bin column b of window row r: the lower window bounds of the
    // tile's eight node columns (b < 8), then their upper bounds
    __shared__ int32_t s_st[MB_ROWS][16];
    const int tid = threadIdx.x;
    const int lane = tid & 3;
    const int64_t tile = blockIdx.x;
    const SetDesc& sd = wv.sets[set_search(wv.S, tile, [&](int s) { return wv.sets[s].t0; })];
    const MeshD m = sd.m;
    const Grid g = sd.g;
    const int32_t* start = wv.start + sd.b0;
    // the union of the tile's node windows, in bins
    int tx, ty;
    tile_xy(sd, static_cast<int>(tile - sd.t0), tx, ty);
    const int i0 = 8 * tx;
    auto col_lo = [&](int i) { return max((i - 1) * g.kb - 1, 0); };
    auto col_hi = [&](int i) { return min((i + 1) * g.kb + 1, g.nbx); };
    const int wx0 = col_lo(i0), wx1 = col_hi(i0 + 7);
    const int wy0 = max((8 * ty - 1) * g.kb - 1, 0), wy1 = min((8 * ty + 8) * g.kb + 1, g.nby);
    const int nrow = wy1 - wy0;
    // cell codes n00 * 2 + lower need the set's nodes below 2^30
    bool staged = nrow <= MB_ROWS && static_cast<int64_t>(m.nx + 1) * (m.ny + 1) < (int64_t(1) << 30);
    if (staged) {
        // the bounds of every node window in every window row, and the rows'
        // lengths prefixed (the first wave, one row a lane)
        for (int e = tid; e < nrow * 16; e += 256) {
            const int r = e >> 4, b = e & 15;
            const int i = i0 + (b & 7);
            s_st[r][b] = start[(wy0 + r) * g.nbx + (b < 8 ? col_lo(i) : col_hi(i))];
        }
        int len = 0;
        if (tid < nrow) {
            const int row = (wy0 + tid) * g.nbx;
            len = start[row + wx1] - start[row + wx0];
        }
        int inc = len;
#pragma unroll
        for (int d = 1; d < MB_WAVE; d <<= 1) {
            const int o = __shfl_up(inc, d);
            if ((tid & (MB_WAVE - 1)) >= d) inc += o;
        }
        if (tid < MB_WAVE) s_off[tid + 1] = inc;
        if (tid == 0) s_off[0] = 0;
        __syncthreads();
        staged = s_off[nrow] <= MB_CAP;  // uniform over the block
    }
    if (staged) {
        // every particle of the window located once; a thread's particles
        // have all their loads in flight before the first is located
        const int total = s_off[nrow];
        int64_t sp[MB_PT];
#pragma unroll
        for (int k = 0; k < MB_PT; ++k) {
            const int f = tid + 256 * k;
            int lo = 0, hi = nrow - 1;  // the row holding f
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= f) lo = mid;
                else hi = mid - 1;
            }
            sp[k] = f < total ? s_st[lo][0] + (f - s_off[lo]) : -1;
        }
        double2 pp[MB_PT];
        int32_t uu[MB_PT];
#pragma unroll
        for (int k = 0; k < MB_PT; ++k) {
            pp[k] = wv.pos_s[sp[k] >= 0 ? sp[k] : 0];
            uu[k] = wv.perm[sp[k] >= 0 ? sp[k] : 0];
        }
#pragma unroll
        for (int k = 0; k < MB_PT; ++k) {
            const int f = tid + 256 * k;
            if (f >= total) continue;
            const Cell c = cell_of(m, pp[k]);
            s_xi[f] = c.xi;
            s_eta[f] = c.eta;
            s_code[f] = c.ok ? static_cast<int32_t>(c.n00 * 2 + (c.lower ? 1 : 0)) : -1;
            s_uid[f] = uu[k];
        }
        __syncthreads();
    }
    const int64_t slot = tile * TILE_N + (tid >> 2);
    int i, j;
    if (!slot_ij(sd, slot, i, j)) return;  // the four lanes of a node leave together
    const int64_t lnode = static_cast<int64_t>(j) * (m.nx + 1) + i;
    const int bx0 = col_lo(i), bx1 = col_hi(i);
    const int by0 = max((j - 1) * g.kb - 1, 0), by1 = min((j + 1) * g.kb + 1, g.nby);
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    auto add = [&](const Loc& L, int64_t u) {
        if (!L.ok) return;
        const double w = L.n0 == lnode ? L.w0 : (L.n1 == lnode ? L.w1 : (L.n2 == lnode ? L.w2 : 0.0));
        if (w == 0.0) return;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < C) acc[c] += w * static_cast<double>(gv[u * C + c]);
    };
    if (staged) {
        const int bl = i - i0;
        for (int by = by0; by < by1; ++by) {
            const int r = by - wy0;
            const int s0 = s_st[r][bl], s1 = s_st[r][8 + bl];
            const int fo = s_off[r] + (s0 - s_st[r][0]);
            for (int s = s0 + lane; s < s1; s += 4) {
                const int f = fo + (s - s0);
                const int code = s_code[f];
                Cell c;
                c.ok = code >= 0;
                c.n00 = code >> 1;
                c.lower = (code & 1) != 0;
                c.xi = s_xi[f];
                c.eta = s_eta[f];
                add(loc_of(m, c), s_uid[f]);
            }
        }
    } else {
        for (int by = by0; by < by1; ++by) {
            const int s0 = start[by * g.nbx + bx0], s1 = start[by * g.nbx + bx1];
            for (int s = s0 + lane; s < s1; s += 4) add(locate_cell(m, wv.pos_s[s]), wv.perm[s]);
        }
    }
    const int64_t node = sd.n0 + lnode;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c < C) {
            double v = acc[c];
            v += lane_xor<4>(v, 1);
            v += lane_xor<4>(v, 2);
            if (lane == (c & 3)) gmesh[node * C + c] = static_cast<TG>(v);
        }
    }
}

template <typename TG>
void launch_m2p_bwd_gather(const WeightsView& wv, const void* gv, int C, void* gmesh, hipStream_t st) {
    const int blocks = static_cast<int>(wv.n_slots / TILE_N);
    const TG* G = static_cast<const TG*>(gv);
    TG* M = static_cast<TG*>(gmesh);
    switch (C) {
        case 1: k_m2p_bwd_gather<TG, 1><<<blocks, 256, 0, st>>>(wv, G, C, M); break;
        case 2: k_m2p_bwd_gather<TG, 2><<<blocks, 256, 0, st>>>(wv, G, C, M); break;
        case 3: k_m2p_bwd_gather<TG, 3><<<blocks, 256, 0, st>>>(wv, G, C, M); break;
        case 4: k_m2p_bwd_gather<TG, 4><<<blocks, 256, 0, st>>>(wv, G, C, M); break;
        default: k_m2p_bwd_gather<TG, 0><<<blocks, 256, 0, st>>>(wv, G, C, M); break;
    }
}

}  // namespace

int m2p_backward_binned(const WeightsView& wv, const void* mesh_vals, int C, int dtype, const double* pos,
                        const void* grad_vals, void* grad_mesh, double* grad_pos, hipStream_t st) {
    PhaseTimer _timer(PH_M2P_BWD, st);
    if (grad_mesh) {
        if (dtype == P2M_F64) launch_m2p_bwd_gather<double>(wv, grad_vals, C, grad_mesh, st);
        else launch_m2p_bwd_gather<float>(wv, grad_vals, C, grad_mesh, st);
        P2M_HIP(hipGetLastError());
    }
    if (grad_pos) {
        // the position gradient per particle (its own entry, no atomics)
        const MeshOf m{MeshD{}, wv.sets, wv.S};
        const double2* P = reinterpret_cast<const double2*>(pos);
        double2* GP = reinterpret_cast<double2*>(grad_pos);
        if (dtype == P2M_F64)
            launch_m2p_bwd<double>(m, static_cast<const double*>(mesh_vals), C, P, wv.N,
                                   static_cast<const double*>(grad_vals), nullptr, GP, st);
        else
            launch_m2p_bwd<float>(m, static_cast<const float*>(mesh_vals), C, P, wv.N,
                                  static_cast<const float*>(grad_vals), nullptr, GP, st);
        P2M_HIP(hipGetLastError());
    }
    return P2M_OK;
}

int m2p(const MeshD& mesh, const SetDesc* sets, int S, int64_t n_nodes, const void* mesh_vals, int C, int dtype,
        const double* pos, int64_t N, void* vals, hipStream_t st, int m2p_ppt) {
    PhaseTimer _timer(PH_M2P, st);
    // (the kernel keeps element offsets of the mesh array in 32 bits)
    if (n_nodes * C >= (int64_t(1) << 31)) {
        set_error("m2p: %lld mesh nodes x %d channels exceed 2^31 elements", static_cast<long long>(n_nodes), C);
        return P2M_EINVAL;
    }
    const MeshOf m{mesh, sets, S};
    if (dtype == P2M_F64)
        launch_m2p<double, double>(m, mesh_vals, C, pos, N, vals, m2p_ppt, st);
    else if (dtype == P2M_F32)
        launch_m2p<float, float>(m, mesh_vals, C, pos, N, vals, m2p_ppt, st);
    else
        launch_m2p<float, uint16_t>(m, mesh_vals, C, pos, N, vals, m2p_ppt, st);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int m2p_qcsf(const MeshD& m, const int32_t* idx, const double* coef, const void* mesh_vals, int C, int dtype,
             const double* pos, int64_t N, void* vals, hipStream_t st, bool periodic) {
    PhaseTimer _timer(PH_M2P, st);
    const int per = periodic ? 1 : 0;
    if (dtype == P2M_F64)
        per ? launch_m2p_qcsf<double, double, true>(m, idx, coef, mesh_vals, C, pos, N, vals, st)
            : launch_m2p_qcsf<double, double, false>(m, idx, coef, mesh_vals, C, pos, N, vals, st);
    else if (dtype == P2M_F32)
        per ? launch_m2p_qcsf<float, float, true>(m, idx, coef, mesh_vals, C, pos, N, vals, st)
            : launch_m2p_qcsf<float, float, false>(m, idx, coef, mesh_vals, C, pos, N, vals, st);
    else
        per ? launch_m2p_qcsf<float, uint16_t, true>(m, idx, coef, mesh_vals, C, pos, N, vals, st)
            : launch_m2p_qcsf<float, uint16_t, false>(m, idx, coef, mesh_vals, C, pos, N, vals, st);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int m2p_backward(const MeshD& mesh, const SetDesc* sets, int S, int64_t n_nodes, const void* mesh_vals, int C,
                 int dtype, const double* pos, int64_t N, const void* grad_vals, void* grad_mesh, double* grad_pos,
                 hipStream_t st) {
    PhaseTimer _timer(PH_M2P_BWD, st);
    const int64_t nn = n_nodes;
    const MeshOf m{mesh, sets, S};
    const double2* P = reinterpret_cast<const double2*>(pos);
    double2* GP = reinterpret_cast<double2*>(grad_pos);
    if (dtype == P2M_F64) {
        if (grad_mesh) {
            int rc = fill_bytes_zero(grad_mesh, sizeof(double) * nn * C, st);
            if (rc) return rc;
        }
        launch_m2p_bwd<double>(m, static_cast<const double*>(mesh_vals), C, P, N,
                               static_cast<const double*>(grad_vals), static_cast<double*>(grad_mesh), GP, st);
    } else {
        if (grad_mesh) {
            int rc = fill_bytes_zero(grad_mesh, sizeof(float) * nn * C, st);
            if (rc) return rc;
        }
        launch_m2p_bwd<float>(m, static_cast<const float*>(mesh_vals), C, P, N,
                              static_cast<const float*>(grad_vals), static_cast<float*>(grad_mesh), GP, st);
    }
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
