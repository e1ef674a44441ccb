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
// A quad of lanes per node (the forward's layout, k_build_bwd); every
// support entry ends with one pair of atomics on grad_pos.
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
#include <type_traits>

#include "algebra.h"
#include "kernels.h"

namespace p2m {

namespace {

struct BArgs {
    WeightsView w;
    const double2* pos;
    const double* gw;
    double2* gpos;
    int per;  // periodic box: support positions are the nearest images
};

// ---- rows solved by Cholesky: a quad of four lanes per node, nodes in the
// 8 x 8 tiles of the forward's weights pass.  Lanes 0..2 each redo one edge
// system as the forward solved it (same frame: the edge midpoint and length;
// moments, Cholesky with reciprocal pivots, one refinement step), then
// z = G^-1 M Abar and sum_mu wbar_mu A_mu; a closure row's one system is
// computed by all four lanes (strided passes, quad sums), as in the forward.
// Each lane then differentiates the support entries it owns (entry k by
// lane k % 4) with every system's y, z and frame broadcast within the quad:
// Mbar_k = y Abar_k - z A_k - y (z . p_k), chained through the monomials
// p_k of the frame (whose centre and scale are held fixed: the solution does
// not depend on them).  The edge ends also get the derivative through the
// right-hand side -d d^t / 2, and the triangle's vertices the barycentric
// part.  Every owned entry ends with one pair of atomics on grad_pos, or,
// for a handle with a particle-major index, one store of its derivative
// (summed per particle afterwards).
constexpr int QL = 4;
constexpr int QWG = 256;
constexpr int QPB = QWG / QL;
constexpr int SK = 16;       // support entries staged in LDS per node
constexpr int SKP = SK + 1;  // LDS row pitch (distinct banks across quads)
constexpr int MSE = KMAX / QL;

// Value of v in lane L of the quad (DPP quad permute, no LDS round trip).
template <int L>
__device__ __forceinline__ double quad_bcast(double v) {
    constexpr int ctrl = L | (L << 2) | (L << 4) | (L << 6);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double quad_sum(double v) {
    v += lane_xor<QL>(v, 1);
    v += lane_xor<QL>(v, 2);
    return v;
}

// dL/d(position) of a support entry at frame coordinates (x, y) (frame
// scale sc) for the block derivative pbar = dL/dp_k.
__device__ __forceinline__ void chain_monos(const double pbar[6], double x, double y, double sc, double& gx,
                                            double& gy) {
    // d p / dx = (0, 1, 0, 2x, y, 0), d p / dy = (0, 0, 1, 0, x, 2y)
    gx += sc * (pbar[1] + 2.0 * x * pbar[3] + y * pbar[4]);
    gy += sc * (pbar[2] + x * pbar[4] + 2.0 * y * pbar[5]);
}

template <bool PER>
__global__ void __launch_bounds__(QWG) k_build_bwd(BArgs a) {
    __shared__ double2 sp[QPB * SKP];
    __shared__ double sw[QPB * SKP];
    __shared__ uint32_t sm[QPB * SKP];
    const int lane = threadIdx.x & (QL - 1);
    const int qi = threadIdx.x / QL;
    const int64_t tile = blockIdx.x;
    const SetDesc& sd = a.w.sets[set_search(a.w.S, tile, [&](int s) { return a.w.sets[s].t0; })];
    const int64_t slot = tile * TILE_N + qi;
    int i, j;
    const bool valid = slot_ij(sd, slot, i, j);
    const uint32_t meta = valid ? a.w.meta[slot] : 0u;
    const uint32_t type = meta_type(meta);
    const int n = valid ? row_len(meta) : 0;
    const bool inter = valid && n > 0 && !(meta_flags(meta) & MF_SVD) && type == NT_INTERIOR;
    const bool clos = valid && n > 0 && !(meta_flags(meta) & MF_SVD) && (type == NT_RING || type == NT_OUTSIDE);
    const bool act = inter || clos;
    const int64_t node = valid ? ij_node(sd, i, j) : 0;
    const int64_t nn = a.w.n_nodes, ns = a.w.n_slots;
    const double2 q = node_at(sd.m, i, j, PER);
    auto img = [&](double2 p) { return PER ? image_near(sd.m, p, q) : p; };
    // stage the first SK entries: position (image), wbar, ring bits
    const int nst = act ? min(n, SK) : 0;
#pragma unroll
    for (int s = 0; s < SK / QL; ++s) {
        const int k = s * QL + lane;
        if (k < nst) {
            const int64_t u = a.w.idx[k * ns + slot];
            sp[qi * SKP + k] = img(a.pos[u]);
            sw[qi * SKP + k] = a.gw[k * nn + node];
            sm[qi * SKP + k] = a.w.mem[k * ns + slot];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    auto P = [&](int k) -> double2 { return k < SK ? sp[qi * SKP + k] : img(a.pos[a.w.idx[k * ns + slot]]); };
    auto W = [&](int k) -> double { return k < SK ? sw[qi * SKP + k] : a.gw[k * nn + node]; };
    auto Mb = [&](int k) -> uint32_t { return k < SK ? sm[qi * SKP + k] : a.w.mem[k * ns + slot]; };

    double gx[MSE], gy[MSE];  // owned entries k = s * QL + lane
#pragma unroll
    for (int s = 0; s < MSE; ++s) gx[s] = gy[s] = 0.0;
    double tvx[3] = {0.0, 0.0, 0.0}, tvy[3] = {0.0, 0.0, 0.0};  // extra terms of T's vertices
    int lt[3] = {-1, -1, -1};
    int skipped = 0;
    if (inter) {
#pragma unroll
        for (int k = 0; k < 3; ++k) lt[k] = static_cast<int>(meta_t(meta, k));
        const double2 P0 = P(lt[0]), P1 = P(lt[1]), P2 = P(lt[2]);
        const double D = (P1.x - P0.x) * (P2.y - P0.y) - (P1.y - P0.y) * (P2.x - P0.x);
        const double phi[3] = {((P1.x - q.x) * (P2.y - q.y) - (P1.y - q.y) * (P2.x - q.x)) / D,
                               ((q.x - P0.x) * (P2.y - P0.y) - (q.y - P0.y) * (P2.x - P0.x)) / D,
                               ((P1.x - P0.x) * (q.y - P0.y) - (P1.y - P0.y) * (q.x - P0.x)) / D};
        // phase 1: lane e < 3 redoes edge system e
        double y[6] = {0, 0, 0, 0, 0, 0}, z[6] = {0, 0, 0, 0, 0, 0};
        double cx = 0.0, cy = 0.0, sc = 1.0, sa = 0.0;
        int ok = 1;
        if (lane < 3) {
            const int pb = lane == 2 ? 0 : lane + 1;
            const double2 rn = lane == 0 ? P0 : (lane == 1 ? P1 : P2);
            const double2 rs = pb == 0 ? P0 : (pb == 1 ? P1 : P2);
            cx = 0.5 * (rn.x + rs.x);
            cy = 0.5 * (rn.y + rs.y);
            const double dxv = rn.x - rs.x, dyv = rn.y - rs.y;
            sc = 1.0 / sqrt(dxv * dxv + dyv * dyv);
            const uint32_t mask = (1u << lane) | (1u << pb);
            const double pa_ = lane == 0 ? phi[0] : (lane == 1 ? phi[1] : phi[2]);
            const double pb_ = pb == 0 ? phi[0] : (pb == 1 ? phi[1] : phi[2]);
            const double coef = 2.0 * pa_ * pb_;
            const double dx = dxv * sc, dy = dyv * sc;
            const double b[6] = {0.0, 0.0, 0.0, -0.5 * dx * dx, -0.5 * dx * dy, -0.5 * dy * dy};
            Moments mo;
            mo.zero();
            for (int k = 0; k < n; ++k) {
                if (!(Mb(k) & mask)) continue;
                const double2 p = P(k);
                mo.add((p.x - cx) * sc, (p.y - cy) * sc);
            }
            double L[6][6];
            mo.gram(L);
            ok = chol6(L) ? 1 : 0;
            if (ok) {
                chol6_solve(L, b, y);
                double r[6] = {0, 0, 0, 0, 0, 0};
                for (int k = 0; k < n; ++k) {
                    if (!(Mb(k) & mask)) continue;
                    const double2 p = P(k);
                    double pm[6];
                    monos((p.x - cx) * sc, (p.y - cy) * sc, pm);
                    const double A = dot6(pm, y);
#pragma unroll
                    for (int t = 0; t < 6; ++t) r[t] += A * pm[t];
                }
#pragma unroll
                for (int t = 0; t < 6; ++t) r[t] = b[t] - r[t];
                double d[6];
                chol6_solve(L, r, d);
#pragma unroll
                for (int t = 0; t < 6; ++t) y[t] += d[t];
                // v = M Abar (Abar_k = coef wbar_k) and sum_k wbar_k A_k
                double v[6] = {0, 0, 0, 0, 0, 0};
                for (int k = 0; k < n; ++k) {
                    if (!(Mb(k) & mask)) continue;
                    const double2 p = P(k);
                    double pm[6];
                    monos((p.x - cx) * sc, (p.y - cy) * sc, pm);
                    const double wk = W(k);
                    sa += wk * dot6(pm, y);
                    const double ab = coef * wk;
#pragma unroll
                    for (int t = 0; t < 6; ++t) v[t] += ab * pm[t];
                }
                chol6_solve(L, v, z);
            } else {
                // (the forward's Cholesky accepted this system with a wide
                // margin, so this does not happen; counted if it does)
#pragma unroll
                for (int t = 0; t < 6; ++t) y[t] = z[t] = 0.0;
                skipped = 1;
            }
        }
        // phase 2: every lane differentiates its own entries
        double phib[3] = {W(lt[0]), W(lt[1]), W(lt[2])};
        auto edge = [&](auto E) {
            constexpr int e = decltype(E)::value;
            constexpr int pa = e, pb = e == 2 ? 0 : e + 1;
            double ye[6], ze[6];
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                ye[t] = quad_bcast<e>(y[t]);
                ze[t] = quad_bcast<e>(z[t]);
            }
            const double cxe = quad_bcast<e>(cx), cye = quad_bcast<e>(cy), sce = quad_bcast<e>(sc);
            const double sae = quad_bcast<e>(sa);
            const double coef = 2.0 * phi[pa] * phi[pb];
            phib[pa] += 2.0 * phi[pb] * sae;
            phib[pb] += 2.0 * phi[pa] * sae;
            constexpr uint32_t mask = (1u << pa) | (1u << pb);
#pragma unroll
            for (int s = 0; s < MSE; ++s) {
                const int k = s * QL + lane;
                if (k >= n || !(Mb(k) & mask)) continue;
                const double2 p = P(k);
                const double x = (p.x - cxe) * sce, yy = (p.y - cye) * sce;
                double pm[6];
                monos(x, yy, pm);
                const double A = dot6(pm, ye), zp = dot6(ze, pm), ab = coef * W(k);
                double pbar[6];
#pragma unroll
                for (int t = 0; t < 6; ++t) pbar[t] = ye[t] * ab - ze[t] * A - ye[t] * zp;
                chain_monos(pbar, x, yy, sce, gx[s], gy[s]);
            }
            // right-hand side: b = (0, 0, 0, -dx^2/2, -dx dy/2, -dy^2/2), d = (r_nu - r_sigma) sc
            const double2 rn = pa == 0 ? P0 : (pa == 1 ? P1 : P2);
            const double2 rs = pb == 0 ? P0 : (pb == 1 ? P1 : P2);
            const double dx = (rn.x - rs.x) * sce, dy = (rn.y - rs.y) * sce;
            const double ddx = -ze[3] * dx - 0.5 * ze[4] * dy;
            const double ddy = -0.5 * ze[4] * dx - ze[5] * dy;
            tvx[pa] += ddx * sce;
            tvy[pa] += ddy * sce;
            tvx[pb] -= ddx * sce;
            tvy[pb] -= ddy * sce;
        };
        edge(std::integral_constant<int, 0>{});
        edge(std::integral_constant<int, 1>{});
        edge(std::integral_constant<int, 2>{});
        // barycentric coordinates
        const double e1x = P1.x - P0.x, e1y = P1.y - P0.y, e2x = P2.x - P0.x, e2y = P2.y - P0.y;
        const double f1 = phib[1] - phib[0], f2 = phib[2] - phib[0];
        const double lx = (f1 * e2y - f2 * e1y) / D;
        const double ly = (-f1 * e2x + f2 * e1x) / D;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            tvx[k] -= phi[k] * lx;
            tvy[k] -= phi[k] * ly;
        }
        skipped += lane_xor<QL>(skipped, 1);
        skipped += lane_xor<QL>(skipped, 2);
    } else if (clos) {
        // weights = M^t y with G y = p(q), the forward's frame: centroid of the
        // nearest particles, RMS radius; passes shared by the four lanes
        auto each4 = [&](auto&& f) {
            for (int k = lane; k < nst; k += QL) f(k, sp[qi * SKP + k]);
            for (int k = SK + lane; k < n; k += QL) f(k, P(k));
        };
        double sx = 0.0, sy = 0.0;
        each4([&](int, double2 p) {
            sx += p.x;
            sy += p.y;
        });
        const double cx = quad_sum(sx) / n, cy = quad_sum(sy) / n;
        double r2 = 0.0;
        each4([&](int, double2 p) { r2 += (p.x - cx) * (p.x - cx) + (p.y - cy) * (p.y - cy); });
        r2 = quad_sum(r2);
        const double sc = r2 > 0.0 ? 1.0 / sqrt(r2 / n) : 1.0;
        Moments mo;
        mo.zero();
        each4([&](int, double2 p) { mo.add((p.x - cx) * sc, (p.y - cy) * sc); });
#pragma unroll
        for (int t = 0; t < 15; ++t) mo.m[t] = quad_sum(mo.m[t]);
        double b[6];
        monos((q.x - cx) * sc, (q.y - cy) * sc, b);
        double L[6][6];
        mo.gram(L);
        if (chol6(L)) {
            double y[6], z[6];
            chol6_solve(L, b, y);
            double r[6] = {0, 0, 0, 0, 0, 0}, v[6] = {0, 0, 0, 0, 0, 0};
            each4([&](int, double2 p) {
                double pm[6];
                monos((p.x - cx) * sc, (p.y - cy) * sc, pm);
                const double A = dot6(pm, y);
#pragma unroll
                for (int t = 0; t < 6; ++t) r[t] += A * pm[t];
            });
#pragma unroll
            for (int t = 0; t < 6; ++t) r[t] = b[t] - quad_sum(r[t]);
            double d[6];
            chol6_solve(L, r, d);
#pragma unroll
            for (int t = 0; t < 6; ++t) y[t] += d[t];
            each4([&](int k, double2 p) {
                double pm[6];
                monos((p.x - cx) * sc, (p.y - cy) * sc, pm);
                const double wk = W(k);
#pragma unroll
                for (int t = 0; t < 6; ++t) v[t] += wk * pm[t];
            });
#pragma unroll
            for (int t = 0; t < 6; ++t) v[t] = quad_sum(v[t]);
            chol6_solve(L, v, z);
#pragma unroll
            for (int s = 0; s < MSE; ++s) {
                const int k = s * QL + lane;
                if (k >= n) continue;
                const double2 p = P(k);
                const double x = (p.x - cx) * sc, yy = (p.y - cy) * sc;
                double pm[6];
                monos(x, yy, pm);
                const double A = dot6(pm, y), zp = dot6(z, pm), ab = W(k);
                double pbar[6];
#pragma unroll
                for (int t = 0; t < 6; ++t) pbar[t] = y[t] * ab - z[t] * A - y[t] * zp;
                chain_monos(pbar, x, yy, sc, gx[s], gy[s]);
            }
        } else {
            skipped = 1;
        }
    }
    if (act) {
#pragma unroll
        for (int s = 0; s < MSE; ++s) {
            const int k = s * QL + lane;
            if (k >= n) continue;
            double ax = gx[s], ay = gy[s];
#pragma unroll
            for (int t = 0; t < 3; ++t)
                if (k == lt[t]) {
                    ax += tvx[t];
                    ay += tvy[t];
                }
            if (a.w.gent) {
                // (rows of this kernel are at most KMAX long)
                a.w.gent[k * ns + slot] = make_double2(ax, ay);
            } else {
                const int64_t u = a.w.idx[k * ns + slot];
                atomicAdd(&a.gpos[u].x, ax);
                atomicAdd(&a.gpos[u].y, ay);
            }
        }
        if (lane == 0 && skipped) atomicAdd(&a.w.diag[D_BWDSKIP], static_cast<unsigned long long>(skipped));
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
        const int64_t slot = static_cast<int64_t>(static_cast<uint32_t>(a.w.rd[li]) & ~RD_SOLVED);
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
            // entries KMAX.. of a long row live in its overflow row
            const bool main = lane < KMAX;
            const int64_t at = main ? lane * ns + slot : ovf_at(a.w.n_ovf, a.w.orow[slot], lane);
            u = main ? a.w.idx[at] : a.w.oidx[at];
            const double2 r = a.pos[u];
            p = per ? image_near(sd.m, r, q) : r;
            wb = a.gw[lane * nn + node];
            bits = main ? a.w.mem[at] : a.w.omem[at];
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
            if (a.w.gent) {
                const int32_t orow = n > KMAX ? a.w.orow[slot] : 0;
                a.w.gent[entry_at(ns, a.w.n_ovf, orow, slot, lane)] = make_double2(gx, gy);
            } else {
                atomicAdd(&a.gpos[u].x, gx);
                atomicAdd(&a.gpos[u].y, gy);
            }
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
    const int32_t r = n > KMAX ? w.orow[slot] : 0;
    for (int k = 0; k < KROW; ++k) {
        const bool main = k < KMAX;
        const int64_t at = main ? k * ns + slot : ovf_at(w.n_ovf, r, k);
        if (idx) idx[k * nn + node] = k < n ? (main ? w.idx[at] : w.oidx[at]) : -1;
        if (wts) wts[k * nn + node] = k < n ? (main ? w.w64[at] : w.ow64[at]) : 0.0;
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
    // a block per 8 x 8 node tile (the forward's tiles), a quad per node
    const int blocks = static_cast<int>(w.n_slots / TILE_N);
    if (periodic) k_build_bwd<true><<<blocks, QWG, 0, st>>>(a);
    else k_build_bwd<false><<<blocks, QWG, 0, st>>>(a);
    P2M_HIP(hipGetLastError());
    // rows of the rank-revealing solver (normally none; the grid loops over
    // the list)
    k_build_bwd_svd<<<16, 256, 0, st>>>(a);
    P2M_HIP(hipGetLastError());
    // a particle-major index: the per-entry derivatives summed per particle
    if (w.gent) return gather_entry_grads(w, grad_pos, st);
    return P2M_OK;
}

int export_weights(const WeightsView& w, int32_t* idx, double* wts, int32_t* cnt, int32_t* tri, hipStream_t st) {
    const int blocks = static_cast<int>((w.n_nodes + 255) / 256);
    k_export<<<blocks, 256, 0, st>>>(w, idx, wts, cnt, tri);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
