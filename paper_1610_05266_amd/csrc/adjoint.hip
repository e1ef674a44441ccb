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
//
// Rows the forward solved with the rank-revealing solver (flag MF_SVD) are
// differentiated by a second kernel, one wave per row, from the SVD of each
// system: for a full-rank system the formula above with G^-1 = V S^-2 V^t.
// A system of rank below 6 has least-squares weights that are not
// differentiable where the rank changes (and depend on the frame of its
// conditions): the derivative through its coefficients is left out and
// counted (diag D_BWDSKIP); its part through the barycentric factors is kept.
// Both kernels use the forward's algebra (algebra.h): its Cholesky with
// reciprocal pivots and the same SVD.
#include <cfloat>

#include "algebra.h"
#include "kernels.h"

namespace p2m {

namespace {

constexpr int WG = 64;

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
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j2 = 0; j2 <= i; ++j2) L[i][j2] += p[i] * p[j2];
    }
    if (!chol6(L)) return false;
    chol6_solve(L, b, y);
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
    chol6_solve(L, r, d);
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
    chol6_solve(L, v, z);
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
    if (meta_flags(meta) & MF_SVD) return;  // k_build_bwd_svd
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
            if (!block_backward(n, member, coord, b, abar, addsc, y, bb)) {
                // (the forward's Cholesky accepted this system with a wide
                // margin, so this does not happen; counted if it does)
                atomicAdd(&a.w.diag[D_BWDSKIP], 1ull);
                continue;
            }
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
        if (!block_backward(n, member, coord, b, wbar, addsc, y, bb)) atomicAdd(&a.w.diag[D_BWDSKIP], 1ull);
    }
    for (int k = 0; k < n; ++k) {
        const int64_t u = a.w.idx[k * ns + slot];
        atomicAdd(&a.gpos[u].x, gx[k * WG]);
        atomicAdd(&a.gpos[u].y, gy[k * WG]);
    }
}

// Rows of the rank-revealing solver (listed by the build): one wave per row,
// support entry k in lane k.  Each system is factored exactly as the forward
// factored it (same frame, same SVD), so its coefficients are the forward's.
// For a full-rank system, y = V S^-2 V^t b and z = V S^-2 (B V)^t Abar give
// Mbar = y Abar^t - z A^t - y (z^t M) and bbar = z, chained through the
// condition vectors of the frame (relative to the edge ends, or to the node
// in units of h), whose reference points are held fixed: the solution of a
// full-rank system does not depend on them.
__global__ void __launch_bounds__(256) k_build_bwd_svd(BArgs a) {
    const int lane = threadIdx.x & 63;
    const int count = static_cast<int>(a.w.diag[D_RDCNT]);
    const int waves = static_cast<int>(gridDim.x) * 4;
    const int w0 = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x * 4 + threadIdx.x / 64));
    const int64_t nn = a.w.n_nodes, ns = a.w.n_slots;
    const bool per = a.per != 0;
    for (int li = w0; li < count; li += waves) {
        const int64_t slot = a.w.rd[li];
        const SetDesc& sd = a.w.sets[set_search(a.w.S, slot / TILE_N, [&](int s) { return a.w.sets[s].t0; })];
        int i, j;
        if (!slot_ij(sd, slot, i, j)) continue;
        const int64_t node = ij_node(sd, i, j);
        const uint32_t meta = a.w.meta[slot];
        const uint32_t type = meta_type(meta);
        const uint32_t flags = meta_flags(meta);
        const int n = row_len(meta);
        if (type == NT_FAILED || n == 0 || !(flags & MF_SVD)) continue;
        const double2 q = node_at(sd.m, i, j, per);
        const bool in = lane < n;
        int64_t u = 0;
        double2 p = make_double2(0.0, 0.0);
        double wb = 0.0;
        uint32_t bits = 0;
        if (in) {
            u = a.w.idx[lane * ns + slot];
            const double2 r = a.pos[u];
            p = per ? image_near(sd.m, r, q) : r;
            wb = a.gw[lane * nn + node];
            bits = a.w.mem[lane * ns + slot];
        }
        double gx = 0.0, gy = 0.0;
        int skipped = 0;
        WaveSVD sv;
        // the full-rank adjoint of one factored system, this lane's share:
        // dL/d(condition vector pk) in pbar
        auto adjoint = [&](const double b[6], const double pk[6], double ab, double pbar[6], double z[6]) {
            double c[6], t[6], y[6], uu[6];
            wave_vt(sv, b, lane, c);
#pragma unroll
            for (int k = 0; k < 6; ++k) t[k] = c[k] / (sv.s[k] * sv.s[k]);
            wave_v(sv, t, y);
#pragma unroll
            for (int k = 0; k < 6; ++k) uu[k] = uniform(wave_sum(sv.B[k] * ab)) / (sv.s[k] * sv.s[k]);
            wave_v(sv, uu, z);
            const double Ak = dot6(pk, y), zp = dot6(z, pk);
#pragma unroll
            for (int k = 0; k < 6; ++k) pbar[k] = y[k] * ab - z[k] * Ak - y[k] * zp;
        };
        if (type == NT_INTERIOR) {
            const int lt[3] = {static_cast<int>(meta_t(meta, 0)), static_cast<int>(meta_t(meta, 1)),
                               static_cast<int>(meta_t(meta, 2))};
            double2 P[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) P[k] = make_double2(lane_value(p.x, lt[k]), lane_value(p.y, lt[k]));
            const double D = (P[1].x - P[0].x) * (P[2].y - P[0].y) - (P[1].y - P[0].y) * (P[2].x - P[0].x);
            const double phi[3] = {((P[1].x - q.x) * (P[2].y - q.y) - (P[1].y - q.y) * (P[2].x - q.x)) / D,
                                   ((q.x - P[0].x) * (P[2].y - P[0].y) - (q.y - P[0].y) * (P[2].x - P[0].x)) / D,
                                   ((P[1].x - P[0].x) * (q.y - P[0].y) - (P[1].y - P[0].y) * (q.x - P[0].x)) / D};
            double phib[3] = {lane_value(wb, lt[0]), lane_value(wb, lt[1]), lane_value(wb, lt[2])};
#pragma unroll
            for (int ed = 0; ed < 3; ++ed) {
                const int pa = ed, pb = ed == 2 ? 0 : ed + 1;
                const double2 rn = P[pa], rs = P[pb];
                const double dxv = rn.x - rs.x, dyv = rn.y - rs.y;
                const double is = 1.0 / sqrt(dxv * dxv + dyv * dyv);
                const bool mem = in && (((bits >> pa) & 1u) || ((bits >> pb) & 1u));
                const int keff = __popcll(__ballot(mem));
                const double ax = (p.x - rn.x) * is, ay = (p.y - rn.y) * is;
                const double cx = (p.x - rs.x) * is, cy = (p.y - rs.y) * is;
                double pk[6] = {1.0, ax, ay, ax * cx, 0.5 * (ax * cy + ay * cx), ay * cy};
                if (!mem) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) pk[k] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < 6; ++k) sv.B[k] = pk[k];
                wave_svd(sv, lane, keff);
                const double dx = dxv * is, dy = dyv * is;
                const double b[6] = {0.0, 0.0, 0.0, -0.5 * dx * dx, -0.5 * dx * dy, -0.5 * dy * dy};
                const double A = wave_svd_solve(sv, b, lane);
                // sum_mu wbar_mu A_mu feeds phibar of the two edge ends
                const double sa = uniform(wave_sum(mem ? wb * A : 0.0));
                phib[pa] += 2.0 * phi[pb] * sa;
                phib[pb] += 2.0 * phi[pa] * sa;
                if (flags & (MF_RD0 << ed)) {
                    ++skipped;
                    continue;
                }
                const double coef = 2.0 * phi[pa] * phi[pb];
                double pbar[6], z[6];
                adjoint(b, pk, mem ? coef * wb : 0.0, pbar, z);
                if (mem) {
                    // d pk / dx = (0, 1, 0, a_x + c_x, (a_y + c_y) / 2, 0) / s, likewise y
                    gx += is * (pbar[1] + (ax + cx) * pbar[3] + 0.5 * (ay + cy) * pbar[4]);
                    gy += is * (pbar[2] + 0.5 * (ax + cx) * pbar[4] + (ay + cy) * pbar[5]);
                }
                // right-hand side: d = (r_nu - r_sigma) / s
                const double ddx = -z[3] * dx - 0.5 * z[4] * dy;
                const double ddy = -0.5 * z[4] * dx - z[5] * dy;
                if (lane == lt[pa]) {
                    gx += ddx * is;
                    gy += ddy * is;
                }
                if (lane == lt[pb]) {
                    gx -= ddx * is;
                    gy -= ddy * is;
                }
            }
            // barycentric coordinates
            const double e1x = P[1].x - P[0].x, e1y = P[1].y - P[0].y, e2x = P[2].x - P[0].x, e2y = P[2].y - P[0].y;
            const double f1 = phib[1] - phib[0], f2 = phib[2] - phib[0];
            const double lx = (f1 * e2y - f2 * e1y) / D;
            const double ly = (-f1 * e2x + f2 * e1x) / D;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (lane == lt[k]) {
                    gx -= phi[k] * lx;
                    gy -= phi[k] * ly;
                }
        } else {
            // closure: the monomials of (r - q) / h against p(0)
            const double ih = 1.0 / sd.h;
            const double x = (p.x - q.x) * ih, y = (p.y - q.y) * ih;
            double pk[6];
            monos(x, y, pk);
            if (!in) {
#pragma unroll
                for (int k = 0; k < 6; ++k) pk[k] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) sv.B[k] = pk[k];
            wave_svd(sv, lane, n);
            if (flags & MF_RD0) {
                skipped = 1;
            } else {
                const double b[6] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                double pbar[6], z[6];
                adjoint(b, pk, in ? wb : 0.0, pbar, z);
                if (in) {
                    gx += ih * (pbar[1] + 2.0 * x * pbar[3] + y * pbar[4]);
                    gy += ih * (pbar[2] + x * pbar[4] + 2.0 * y * pbar[5]);
                }
            }
        }
        if (in) {
            atomicAdd(&a.gpos[u].x, gx);
            atomicAdd(&a.gpos[u].y, gy);
        }
        if (lane == 0 && skipped) atomicAdd(&a.w.diag[D_BWDSKIP], static_cast<unsigned long long>(skipped));
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
    // (the count of left-out systems starts at zero for every call: a fill
    // kernel, so that the call can be captured in a graph)
    int rc = fill_u64(w.diag + D_BWDSKIP, 0ull, 1, st);
    if (rc) return rc;
    const int blocks = static_cast<int>((w.n_nodes + WG - 1) / WG);
    k_build_bwd<<<blocks, WG, 0, st>>>(a);
    P2M_HIP(hipGetLastError());
    // rows of the rank-revealing solver (normally none; the grid loops over
    // the list)
    k_build_bwd_svd<<<16, 256, 0, st>>>(a);
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
