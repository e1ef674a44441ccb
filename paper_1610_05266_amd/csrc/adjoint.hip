// Adjoint of the weight build with respect to particle positions, and the
// ELL export used for inspection.
//
// For fixed combinatorics (triangle, rings, nearest sets) the weights of a
// node are smooth functions of the positions of its support.  Reverse mode,
// given wbar = dL/dpsi for the node's ELL row:
//   * barycentric part: phi solves sum_k phi_k P_k = q, sum_k phi_k = 1, so
//     dL/dP_k = -phi_k grad(l), l the linear function taking the values
//     phibar_k at the vertices P_k.
//   * each minimum-norm block A = M^t y, G y = b, G = M M^t (M the 6 x K
//     monomial matrix of the centred, scaled coordinates): with Abar given,
//     z = G^{-1} M Abar, Mbar = y Abar^t - z A^t - y (z^t M), bbar = z.  The
//     centre and scale are held fixed; the solution does not depend on them
//     (eq. A2_2 and the affine invariance of the moment conditions), so this
//     is the exact derivative.
//   * the right-hand side -d d^t / 2 (d the scaled edge vector) of eq. A2_2
//     depends on the two edge ends.
// Contributions are accumulated per support entry in LDS and added to
// grad_pos with one pair of atomics per entry.
#include <cfloat>

#include "kernels.h"

namespace p2m {

namespace {

constexpr int WG = 64;

__device__ __forceinline__ void monos(double x, double y, double p[6]) {
    p[0] = 1.0;
    p[1] = x;
    p[2] = y;
    p[3] = x * x;
    p[4] = x * y;
    p[5] = y * y;
}

__device__ void gram_add(double G[6][6], const double p[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) G[i][j] += p[i] * p[j];
}

__device__ bool chol(double G[6][6]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double djj = G[j][j];
        double d = djj;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= G[j][k] * G[j][k];
        if (!(d > 1e-12 * djj)) return false;
        const double r = sqrt(d);
        G[j][j] = r;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = G[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= G[i][k] * G[j][k];
            G[i][j] = s / r;
        }
    }
    return true;
}

__device__ void csolve(const double L[6][6], const double b[6], double y[6]) {
    double z[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
        z[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = z[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[k][i] * y[k];
        y[i] = s / L[i][i];
    }
}

__device__ __forceinline__ double dot6(const double a[6], const double b[6]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}

struct BArgs {
    WeightsView w;
    const double2* pos;
    const double* gw;
    double2* gpos;
    int per;  // periodic box: support positions are the nearest images
};

// Reverse-mode of one minimum-norm block.  Entries k < n with member(k);
// coord(k, x, y) gives the centred, scaled coordinates, wb(k) the Abar
// weights, and add(k, gx, gy) receives d/d(coords).  b is the right-hand side;
// on return bbar holds z.
template <class Member, class Coord, class Abar, class Add>
__device__ bool block_backward(int n, Member member, Coord coord, const double b[6], Abar abar, Add add,
                               double y[6], double bbar[6]) {
    double L[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) L[i][j] = 0.0;
    for (int k = 0; k < n; ++k) {
        if (!member(k)) continue;
        double x, yy, p[6];
        coord(k, x, yy);
        monos(x, yy, p);
        gram_add(L, p);
    }
    if (!chol(L)) return false;
    csolve(L, b, y);
    // refine y as the forward does
    double r[6] = {b[0], b[1], b[2], b[3], b[4], b[5]};
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < n; ++k) {
        if (!member(k)) continue;
        double x, yy, p[6];
        coord(k, x, yy);
        monos(x, yy, p);
        const double a = dot6(p, y);
#pragma unroll
        for (int i = 0; i < 6; ++i) r[i] -= a * p[i];
    }
    double d[6];
    csolve(L, r, d);
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] += d[i];
    for (int k = 0; k < n; ++k) {
        if (!member(k)) continue;
        double x, yy, p[6];
        coord(k, x, yy);
        monos(x, yy, p);
        const double ab = abar(k);
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] += ab * p[i];
    }
    double z[6];
    csolve(L, v, z);
    for (int k = 0; k < n; ++k) {
        if (!member(k)) continue;
        double x, yy, p[6];
        coord(k, x, yy);
        monos(x, yy, p);
        const double A = dot6(p, y);
        const double zp = dot6(z, p);
        const double ab = abar(k);
        double pb[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) pb[i] = y[i] * ab - z[i] * A - y[i] * zp;
        // d p / dx = (0, 1, 0, 2x, y, 0), d p / dy = (0, 0, 1, 0, x, 2y)
        const double gx = pb[1] + 2.0 * x * pb[3] + yy * pb[4];
        const double gy = pb[2] + x * pb[4] + 2.0 * yy * pb[5];
        add(k, gx, gy);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) bbar[i] = z[i];
    return true;
}

__global__ void __launch_bounds__(WG) k_build_bwd(BArgs a) {
    __shared__ double sgx[KMAX * WG];
    __shared__ double sgy[KMAX * WG];
    const int tid = threadIdx.x;
    const int64_t node = static_cast<int64_t>(blockIdx.x) * WG + tid;
    if (node >= a.w.n_nodes) return;
    const SetDesc& sd = a.w.sets[set_search(a.w.S, node, [&](int s) { return a.w.sets[s].n0; })];
    const MeshD m = sd.m;
    const int stride = m.nx + 1;
    const int64_t ln = node - sd.n0;
    const int i = static_cast<int>(ln % stride), j = static_cast<int>(ln / stride);
    const int64_t slot = node_slot(sd, i, j);
    const uint32_t meta = a.w.meta[slot];
    const uint32_t type = meta_type(meta);
    const int n = row_len(meta);
    if (type == NT_FAILED || n == 0) return;
    const int64_t nn = a.w.n_nodes, ns = a.w.n_slots;
    const bool per = a.per != 0;
    const double2 q = node_at(m, i, j, per);
    double* gx = sgx + tid;
    double* gy = sgy + tid;
    for (int k = 0; k < n; ++k) {
        gx[k * WG] = 0.0;
        gy[k * WG] = 0.0;
    }
    // (an image moves with its particle: its derivative is the particle's)
    auto P = [&](int k) {
        const double2 p = a.pos[a.w.idx[k * ns + slot]];
        return per ? image_near(m, p, q) : p;
    };
    auto wbar = [&](int k) { return a.gw[k * nn + node]; };
    auto add = [&](int k, double dx, double dy) {
        gx[k * WG] += dx;
        gy[k * WG] += dy;
    };

    if (type == NT_INTERIOR) {
        const int lt[3] = {static_cast<int>(meta_t(meta, 0)), static_cast<int>(meta_t(meta, 1)),
                           static_cast<int>(meta_t(meta, 2))};
        const double2 P0 = P(lt[0]), P1 = P(lt[1]), P2 = P(lt[2]);
        const double D = (P1.x - P0.x) * (P2.y - P0.y) - (P1.y - P0.y) * (P2.x - P0.x);
        const double phi[3] = {((P1.x - q.x) * (P2.y - q.y) - (P1.y - q.y) * (P2.x - q.x)) / D,
                               ((q.x - P0.x) * (P2.y - P0.y) - (q.y - P0.y) * (P2.x - P0.x)) / D,
                               ((P1.x - P0.x) * (q.y - P0.y) - (P1.y - P0.y) * (q.x - P0.x)) / D};
        double phib[3] = {wbar(lt[0]), wbar(lt[1]), wbar(lt[2])};
        for (int e = 0; e < 3; ++e) {
            const int pa = e, pb = (e + 1) % 3;
            const double2 rn = P(lt[pa]), rs = P(lt[pb]);
            const double cxm = 0.5 * (rn.x + rs.x), cym = 0.5 * (rn.y + rs.y);
            const double dxv = rn.x - rs.x, dyv = rn.y - rs.y;
            const double is = 1.0 / sqrt(dxv * dxv + dyv * dyv);
            const int mask = (1 << pa) | (1 << pb);
            auto member = [&](int k) { return (a.w.mem[k * ns + slot] & mask) != 0; };
            auto coord = [&](int k, double& x, double& y) {
                const double2 p = P(k);
                x = (p.x - cxm) * is;
                y = (p.y - cym) * is;
            };
            const double coef = 2.0 * phi[pa] * phi[pb];
            auto abar = [&](int k) { return coef * wbar(k); };
            auto addsc = [&](int k, double dx, double dy) { add(k, dx * is, dy * is); };
            const double dx = dxv * is, dy = dyv * is;
            const double b[6] = {0.0, 0.0, 0.0, -0.5 * dx * dx, -0.5 * dx * dy, -0.5 * dy * dy};
            double y[6], bb[6];
            if (!block_backward(n, member, coord, b, abar, addsc, y, bb)) continue;
            // sum_mu wbar_mu A_mu feeds phibar of the two edge ends
            double sa = 0.0;
            for (int k = 0; k < n; ++k) {
                if (!member(k)) continue;
                double x, yy, p[6];
                coord(k, x, yy);
                monos(x, yy, p);
                sa += wbar(k) * dot6(p, y);
            }
            phib[pa] += 2.0 * phi[pb] * sa;
            phib[pb] += 2.0 * phi[pa] * sa;
            // right-hand side: b = (0,0,0,-dx^2/2,-dx dy/2,-dy^2/2), d = (r_nu - r_sigma) * is
            const double ddx = -bb[3] * dx - 0.5 * bb[4] * dy;
            const double ddy = -0.5 * bb[4] * dx - bb[5] * dy;
            add(lt[pa], ddx * is, ddy * is);
            add(lt[pb], -ddx * is, -ddy * is);
        }
        // barycentric coordinates
        const double e1x = P1.x - P0.x, e1y = P1.y - P0.y, e2x = P2.x - P0.x, e2y = P2.y - P0.y;
        const double f1 = phib[1] - phib[0], f2 = phib[2] - phib[0];
        const double lx = (f1 * e2y - f2 * e1y) / D;
        const double ly = (-f1 * e2x + f2 * e1x) / D;
        for (int k = 0; k < 3; ++k) add(lt[k], -phi[k] * lx, -phi[k] * ly);
    } else {
        // closure node: weights = M^t y with G y = p(q), centroid / RMS scaled
        double mx = 0.0, my = 0.0;
        for (int k = 0; k < n; ++k) {
            const double2 p = P(k);
            mx += p.x;
            my += p.y;
        }
        mx /= n;
        my /= n;
        double r2 = 0.0;
        for (int k = 0; k < n; ++k) {
            const double2 p = P(k);
            r2 += (p.x - mx) * (p.x - mx) + (p.y - my) * (p.y - my);
        }
        const double isc = r2 > 0.0 ? 1.0 / sqrt(r2 / n) : 1.0;
        auto member = [&](int) { return true; };
        auto coord = [&](int k, double& x, double& y) {
            const double2 p = P(k);
            x = (p.x - mx) * isc;
            y = (p.y - my) * isc;
        };
        auto addsc = [&](int k, double dx, double dy) { add(k, dx * isc, dy * isc); };
        double b[6];
        monos((q.x - mx) * isc, (q.y - my) * isc, b);
        double y[6], bb[6];
        block_backward(n, member, coord, b, wbar, addsc, y, bb);
    }
    for (int k = 0; k < n; ++k) {
        const int64_t u = a.w.idx[k * ns + slot];
        atomicAdd(&a.gpos[u].x, gx[k * WG]);
        atomicAdd(&a.gpos[u].y, gy[k * WG]);
    }
}

__global__ void __launch_bounds__(256) k_export(WeightsView w, int32_t* __restrict__ idx, double* __restrict__ wts,
                                                int32_t* __restrict__ cnt, int32_t* __restrict__ tri) {
    const int64_t node = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (node >= w.n_nodes) return;
    const SetDesc& sd = w.sets[set_search(w.S, node, [&](int s) { return w.sets[s].n0; })];
    const int64_t ln = node - sd.n0;
    const int64_t slot = node_slot(sd, static_cast<int>(ln % (sd.m.nx + 1)), static_cast<int>(ln / (sd.m.nx + 1)));
    const uint32_t meta = w.meta[slot];
    const int n = row_len(meta);
    const int64_t nn = w.n_nodes, ns = w.n_slots;
    for (int k = 0; k < KMAX; ++k) {
        if (idx) idx[k * nn + node] = k < n ? w.idx[k * ns + slot] : -1;
        if (wts) wts[k * nn + node] = k < n ? w.w64[k * ns + slot] : 0.0;
    }
    if (cnt) cnt[node] = n;
    if (tri) {
        const bool in = meta_type(meta) == NT_INTERIOR;
        for (int k = 0; k < 3; ++k)
            tri[node * 3 + k] = in ? w.idx[static_cast<int64_t>(meta_t(meta, k)) * ns + slot] : -1;
    }
}

}  // namespace

int build_backward(const WeightsView& w, const double* pos, const double* grad_w, double* grad_pos,
                   hipStream_t st, bool periodic) {
    PhaseTimer _timer(PH_BUILD_BWD, st);
    BArgs a;
    a.w = w;
    a.pos = reinterpret_cast<const double2*>(pos);
    a.gw = grad_w;
    a.gpos = reinterpret_cast<double2*>(grad_pos);
    a.per = periodic ? 1 : 0;
    const int blocks = static_cast<int>((w.n_nodes + WG - 1) / WG);
    k_build_bwd<<<blocks, WG, 0, st>>>(a);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int export_weights(const WeightsView& w, int32_t* idx, double* wts, int32_t* cnt, int32_t* tri, hipStream_t st) {
    const int blocks = static_cast<int>((w.n_nodes + 255) / 256);
    k_export<<<blocks, 256, 0, st>>>(w, idx, wts, cnt, tri);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
