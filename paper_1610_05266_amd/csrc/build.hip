// Weight build: psi_mu(r_i) at every mesh node (App. B of the paper).
//
// One thread per mesh node.  For an interior node q:
//   1. Delaunay triangle T = (a, b, c) of the particles containing q, found by
//      local gift-wrapping: the apex of the Delaunay triangle on one side of a
//      Delaunay edge (v, a) is the candidate that minimises the position of the
//      circumcentre along the edge's bisector (the first particle touched by a
//      circle through v and a growing into that side).  Start from the nearest
//      particle to q, rotate around it to the wedge holding q, then walk
//      (visibility walk) to the triangle containing q.
//   2. The Delaunay rings of a, b and c by rotating around each vertex; their
//      union U (<= P2M_MAX_SUPPORT particles) with membership bits.
//   3. For each edge e = (nu, sigma) of T: the minimum-norm solution of
//      eqs. (A0), (A1), (A2_2) over S_e = ring(nu) U ring(sigma), computed as
//      A_mu = p(x_mu) . y with G y = b, G = sum_mu p(x_mu) p(x_mu)^t the 6x6
//      Gram matrix of the monomials p = (1, x, y, x^2, xy, y^2) of the
//      centred, scaled coordinates x_mu = (r_mu - (r_nu + r_sigma)/2) / |r_nu - r_sigma|
//      (the solution does not depend on the centre and scale, eq. A2_2).
//      FP64 Cholesky plus one step of iterative refinement whose residual
//      b - sum_mu p_mu A_mu is formed from the monomials, not from G.
//   4. psi_mu(q) = phi_mu + 2 sum_e phi_nu phi_sigma A_{mu e} (eq. phiquad,
//      ordered-pair sum), phi the barycentric coordinates of q in T.
// Nodes on the mesh's outer ring and nodes outside the particles' convex hull
// take the minimum-norm weights of the quadratic moment conditions over their
// P2M_CLOSURE_K nearest particles.
//
// Every Delaunay decision is certified: a triangle is used only if its
// circumdisk lies inside the searched bin region (sides of the region on the
// mesh boundary count as walls: no particle lies beyond them).  Otherwise the
// node is redone with a region of twice the half-width, and finally with all
// particles (where every decision is certified).  Near-ties of the FP64
// predicates (|det| within a forward error bound) are counted and broken by
// the user particle id.
#include <cfloat>
#include <climits>

#include "kernels.h"

namespace p2m {

namespace {

constexpr int WG = 64;
constexpr double EPS = DBL_EPSILON;

enum Result : int { R_OK = 0, R_MORE = 1, R_OUTSIDE = 2, R_FAIL = 3, R_CAP = 4 };

struct Region {
    int bx0, bx1, by0, by1;
    double xlo, xhi, ylo, yhi;
    bool global;
};

__device__ Region make_region(const Grid& g, int cbx, int cby, int hw) {
    Region R;
    R.bx0 = max(cbx - hw, 0);
    R.bx1 = min(cbx + hw, g.nbx);
    R.by0 = max(cby - hw, 0);
    R.by1 = min(cby + hw, g.nby);
    const double m = 1e-9 * g.bw;  // covers the rounding of the bin assignment
    R.xlo = R.bx0 == 0 ? -INFINITY : g.x0 + R.bx0 * g.bw + m;
    R.xhi = R.bx1 == g.nbx ? INFINITY : g.x0 + R.bx1 * g.bw - m;
    R.ylo = R.by0 == 0 ? -INFINITY : g.y0 + R.by0 * g.bw + m;
    R.yhi = R.by1 == g.nby ? INFINITY : g.y0 + R.by1 * g.bw - m;
    R.global = R.bx0 == 0 && R.by0 == 0 && R.bx1 == g.nbx && R.by1 == g.nby;
    return R;
}

__device__ __forceinline__ bool disk_inside(const Region& R, double cx, double cy, double r) {
    r *= 1.0 + 1e-9;
    return cx - r >= R.xlo && cx + r <= R.xhi && cy - r >= R.ylo && cy + r <= R.yhi;
}

struct Ctx {
    const double2* __restrict__ pos;  // sorted positions
    const int32_t* __restrict__ perm;
    const int32_t* __restrict__ start;
    Grid g;
    Region R;
    int neardeg;
};

__device__ __forceinline__ double orient(double2 p, double2 q, double2 r) {
    return (q.x - p.x) * (r.y - p.y) - (q.y - p.y) * (r.x - p.x);
}

// Nearest candidate to (qx, qy) other than `exclude`; ties -> smaller user id.
__device__ int nearest(Ctx& c, double qx, double qy, int exclude, double& d2best) {
    int best = -1;
    int buid = -1;
    d2best = INFINITY;
    for (int by = c.R.by0; by < c.R.by1; ++by) {
        const int row = by * c.g.nbx;
        const int s = c.start[row + c.R.bx0], e = c.start[row + c.R.bx1];
        for (int t = s; t < e; ++t) {
            if (t == exclude) continue;
            const double2 p = c.pos[t];
            const double dx = p.x - qx, dy = p.y - qy;
            const double d2 = dx * dx + dy * dy;
            if (d2 < d2best) {
                best = t;
                d2best = d2;
                buid = -1;
            } else if (d2 == d2best) {
                if (buid < 0) buid = c.perm[best];
                const int u = c.perm[t];
                if (u < buid) {
                    best = t;
                    buid = u;
                }
            }
        }
    }
    return best;
}

// Apex of the Delaunay triangle on side `sgn` (+1 left, -1 right) of the
// directed edge v -> a, among the region's candidates: the candidate b with
// sgn*cross(a-v, b-v) > 0 minimising t_b = |B|^2 - A.B over 2 sgn cross(A, B),
// the bisector coordinate of the circumcentre of (v, a, b).  Returns -1 when
// no candidate lies strictly on that side.  (cx, cy, rr): circumcircle.
__device__ int wrap(Ctx& c, int iv, double2 v, int ia, double2 a, double sgn, double& cx, double& cy,
                    double& rr) {
    const double Ax = a.x - v.x, Ay = a.y - v.y;
    const double aAx = fabs(Ax), aAy = fabs(Ay);
    int best = -1, buid = -1;
    double bn = 0.0, bc = 1.0, bN = 0.0, bC = 0.0;
    for (int by = c.R.by0; by < c.R.by1; ++by) {
        const int row = by * c.g.nbx;
        const int s = c.start[row + c.R.bx0], e = c.start[row + c.R.bx1];
        for (int t = s; t < e; ++t) {
            if (t == iv || t == ia) continue;
            const double2 b = c.pos[t];
            const double Bx = b.x - v.x, By = b.y - v.y;
            const double cr = sgn * (Ax * By - Ay * Bx);
            const double Cm = aAx * fabs(By) + aAy * fabs(Bx);
            if (cr <= 4.0 * EPS * Cm) {
                if (cr > -4.0 * EPS * Cm) ++c.neardeg;  // (nearly) on the line through v, a
                continue;
            }
            const double num = Bx * (Bx - Ax) + By * (By - Ay);
            const double Nm = Bx * Bx + By * By + fabs(Bx * Ax) + fabs(By * Ay);
            if (best < 0) {
                best = t;
                bn = num;
                bc = cr;
                bN = Nm;
                bC = Cm;
                buid = -1;
                continue;
            }
            const double lhs = num * bc, rhs = bn * cr;
            const double err = 16.0 * EPS * (Nm * bC + bN * Cm);
            bool take = lhs < rhs - err;
            if (!take && lhs <= rhs + err) {  // co-circular within rounding
                ++c.neardeg;
                if (buid < 0) buid = c.perm[best];
                const int u = c.perm[t];
                take = u < buid;
                if (take) buid = u;
            } else if (take) {
                buid = -1;
            }
            if (take) {
                best = t;
                bn = num;
                bc = cr;
                bN = Nm;
                bC = Cm;
            }
        }
    }
    if (best >= 0) {
        const double tk = bn / (2.0 * bc);
        const double ox = 0.5 * Ax - sgn * tk * Ay;
        const double oy = 0.5 * Ay + sgn * tk * Ax;
        cx = v.x + ox;
        cy = v.y + oy;
        rr = sqrt(ox * ox + oy * oy);
    }
    return best;
}

// Triangle containing q, as sorted indices (CCW).  R_OUTSIDE when q is
// outside the convex hull (only concluded with the global region).
__device__ int locate(Ctx& c, double2 q, int T[3]) {
    double d2;
    const int n0 = nearest(c, q.x, q.y, -1, d2);
    if (n0 < 0) return R_MORE;
    if (!disk_inside(c.R, q.x, q.y, sqrt(d2))) return R_MORE;
    const double2 v = c.pos[n0];
    double e2;
    const int a0 = nearest(c, v.x, v.y, n0, e2);
    if (a0 < 0) return c.R.global ? R_OUTSIDE : R_MORE;
    // the nearest neighbour of v is a Delaunay neighbour of v
    if (!disk_inside(c.R, v.x, v.y, sqrt(e2))) return R_MORE;
    double cx, cy, rr;
    int ta = -1, tb = -1, tcc = -1;
    bool found = false;
    bool open = false;
    int cur = a0;
    double2 pc = c.pos[a0];
    for (int step = 0; step < 2 * KMAX; ++step) {
        const int nx = wrap(c, n0, v, cur, pc, 1.0, cx, cy, rr);
        if (nx < 0) {
            if (!c.R.global) return R_MORE;
            open = true;
            break;
        }
        if (!disk_inside(c.R, cx, cy, rr)) return R_MORE;
        const double2 pn = c.pos[nx];
        if (d2 == 0.0 || (orient(v, pc, q) >= 0.0 && orient(v, pn, q) < 0.0)) {
            ta = n0;
            tb = cur;
            tcc = nx;
            found = true;
            break;
        }
        cur = nx;
        pc = pn;
        if (cur == a0) return R_FAIL;
    }
    if (!found && !open) return R_FAIL;
    if (!found) {
        // v is a hull vertex: rotate clockwise from a0 over the rest of its fan
        cur = a0;
        pc = c.pos[a0];
        for (int step = 0; step < 2 * KMAX; ++step) {
            const int pv = wrap(c, n0, v, cur, pc, -1.0, cx, cy, rr);
            if (pv < 0) {
                if (d2 == 0.0) return R_FAIL;
                return R_OUTSIDE;  // q outside the cone of the open fan
            }
            const double2 pp = c.pos[pv];
            if (d2 == 0.0 || (orient(v, pp, q) >= 0.0 && orient(v, pc, q) < 0.0)) {
                ta = n0;
                tb = pv;
                tcc = cur;
                found = true;
                break;
            }
            cur = pv;
            pc = pp;
        }
        if (!found) return R_FAIL;
    }
    // visibility walk towards q
    for (int step = 0; step < 256; ++step) {
        const double2 pa = c.pos[ta], pb = c.pos[tb], pcc = c.pos[tcc];
        int X, Y;
        if (orient(pb, pcc, q) < 0.0) {
            X = tb;
            Y = tcc;
        } else if (orient(pcc, pa, q) < 0.0) {
            X = tcc;
            Y = ta;
        } else if (orient(pa, pb, q) < 0.0) {
            X = ta;
            Y = tb;
        } else {
            T[0] = ta;
            T[1] = tb;
            T[2] = tcc;
            return R_OK;
        }
        // across edge X -> Y lies the triangle (Y, X, D), D left of Y -> X
        const int D = wrap(c, Y, c.pos[Y], X, c.pos[X], 1.0, cx, cy, rr);
        if (D < 0) return c.R.global ? R_OUTSIDE : R_MORE;
        if (!disk_inside(c.R, cx, cy, rr)) return R_MORE;
        ta = Y;
        tb = X;
        tcc = D;
    }
    return R_FAIL;
}

// Per-thread support list in LDS: sorted particle index | membership << 28.
struct Support {
    int32_t* u;  // [KMAX * WG], entry k of this thread at u[k * WG]
    double* w;   // [KMAX * WG]
    int n;
    __device__ int find(int t) const {
        for (int k = 0; k < n; ++k)
            if ((u[k * WG] & 0x0fffffff) == t) return k;
        return -1;
    }
    __device__ bool add(int t, int bit) {
        for (int k = 0; k < n; ++k) {
            const int e = u[k * WG];
            if ((e & 0x0fffffff) == t) {
                u[k * WG] = e | (bit << 28);
                return true;
            }
        }
        if (n >= KMAX) return false;
        u[n * WG] = t | (bit << 28);
        ++n;
        return true;
    }
    __device__ int idx(int k) const { return u[k * WG] & 0x0fffffff; }
    __device__ int bits(int k) const { return (u[k * WG] >> 28) & 7; }
};

// Ring of T[k] (rotation about T[k] starting with the known triangle T).
__device__ int ring_into(Ctx& c, const int T[3], int k, Support& S) {
    const int v = T[k], first = T[(k + 1) % 3], second = T[(k + 2) % 3];
    const int bit = 1 << k;
    const double2 pv = c.pos[v];
    if (!S.add(first, bit) || !S.add(second, bit)) return R_CAP;
    double cx, cy, rr;
    int cur = second;
    for (int step = 0; step < KMAX; ++step) {
        const int nx = wrap(c, v, pv, cur, c.pos[cur], 1.0, cx, cy, rr);
        if (nx < 0) {
            if (!c.R.global) return R_MORE;
            // open fan (hull vertex): the rest lies clockwise from `first`
            cur = first;
            for (int s2 = 0; s2 < KMAX; ++s2) {
                const int pv2 = wrap(c, v, pv, cur, c.pos[cur], -1.0, cx, cy, rr);
                if (pv2 < 0) return R_OK;
                if (!S.add(pv2, bit)) return R_CAP;
                cur = pv2;
            }
            return R_CAP;
        }
        if (!disk_inside(c.R, cx, cy, rr)) return R_MORE;
        if (nx == first) return R_OK;
        if (!S.add(nx, bit)) return R_CAP;
        cur = nx;
    }
    return R_CAP;
}

// ---------------------------------------------------------------- algebra
__device__ __forceinline__ void monos(double x, double y, double p[6]) {
    p[0] = 1.0;
    p[1] = x;
    p[2] = y;
    p[3] = x * x;
    p[4] = x * y;
    p[5] = y * y;
}

// Accumulate the 15 power sums m_ab = sum x^a y^b (a + b <= 4).
struct Moments {
    double m00, m10, m01, m20, m11, m02, m30, m21, m12, m03, m40, m31, m22, m13, m04;
    __device__ void zero() {
        m00 = m10 = m01 = m20 = m11 = m02 = m30 = m21 = m12 = m03 = m40 = m31 = m22 = m13 = m04 = 0.0;
    }
    __device__ void add(double x, double y) {
        const double x2 = x * x, y2 = y * y, xy = x * y;
        m00 += 1.0;
        m10 += x;
        m01 += y;
        m20 += x2;
        m11 += xy;
        m02 += y2;
        m30 += x2 * x;
        m21 += x2 * y;
        m12 += x * y2;
        m03 += y2 * y;
        m40 += x2 * x2;
        m31 += x2 * xy;
        m22 += x2 * y2;
        m13 += xy * y2;
        m04 += y2 * y2;
    }
    // Gram matrix of p = (1, x, y, x^2, xy, y^2), lower triangle.
    __device__ void gram(double G[6][6]) const {
        G[0][0] = m00;
        G[1][0] = m10; G[1][1] = m20;
        G[2][0] = m01; G[2][1] = m11; G[2][2] = m02;
        G[3][0] = m20; G[3][1] = m30; G[3][2] = m21; G[3][3] = m40;
        G[4][0] = m11; G[4][1] = m21; G[4][2] = m12; G[4][3] = m31; G[4][4] = m22;
        G[5][0] = m02; G[5][1] = m12; G[5][2] = m03; G[5][3] = m22; G[5][4] = m13; G[5][5] = m04;
    }
};

// In-place Cholesky of the lower triangle; false if a pivot is not clearly
// positive (relative threshold on the squared pivot).
__device__ bool chol6(double G[6][6]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double djj = G[j][j];
        double d = djj;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= G[j][k] * G[j][k];
        if (!(d > 1e-12 * djj)) return false;
        const double r = sqrt(d);
        G[j][j] = r;
        const double ir = 1.0 / r;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = G[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= G[i][k] * G[j][k];
            G[i][j] = s * ir;
        }
    }
    return true;
}

__device__ void chol6_solve(const double L[6][6], const double b[6], double y[6]) {
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

// Pseudo-inverse solve by cyclic Jacobi (rank-deficient systems only).
// Eigenvalues below 1e-12 * lambda_max (singular values of the monomial
// matrix below 1e-6 sigma_max) are dropped.
__device__ void pinv6_solve(const double Gl[6][6], const double b[6], double y[6]) {
    double A[6][6], V[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            A[i][j] = i >= j ? Gl[i][j] : Gl[j][i];
            V[i][j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                tot += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < 5; ++p)
            for (int q = p + 1; q < 6; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 6; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 6; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 6; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = cs * vkp - sn * vkq;
                    V[k][q] = sn * vkp + cs * vkq;
                }
            }
    }
    double lmax = 0.0;
    for (int i = 0; i < 6; ++i) lmax = fmax(lmax, A[i][i]);
    double c[6];
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += V[k][i] * b[k];
        c[i] = A[i][i] > 1e-12 * lmax ? s / A[i][i] : 0.0;
    }
    for (int k = 0; k < 6; ++k) {
        double s = 0.0;
        for (int i = 0; i < 6; ++i) s += V[k][i] * c[i];
        y[k] = s;
    }
}

// Minimum-norm solution y of G y = b over the member set; `member(k)` says
// whether support entry k is in the system, `coord(k, x, y)` its centred,
// scaled coordinates.  Returns false when the pseudo-inverse was needed.
template <class Member, class Coord>
__device__ bool min_norm(const Moments& mo, const double b[6], int n, Member member, Coord coord, double y[6]) {
    double L[6][6];
    mo.gram(L);
    double G[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) G[i][j] = L[i][j];
    if (!chol6(L)) {
        pinv6_solve(G, b, y);
        return false;
    }
    chol6_solve(L, b, y);
    // one refinement step with the residual formed from the monomials
    double r[6] = {b[0], b[1], b[2], b[3], b[4], b[5]};
    for (int k = 0; k < n; ++k) {
        if (!member(k)) continue;
        double x, yy;
        coord(k, x, yy);
        double p[6];
        monos(x, yy, p);
        const double a = p[0] * y[0] + p[1] * y[1] + p[2] * y[2] + p[3] * y[3] + p[4] * y[4] + p[5] * y[5];
#pragma unroll
        for (int i = 0; i < 6; ++i) r[i] -= a * p[i];
    }
    double d[6];
    chol6_solve(L, r, d);
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] += d[i];
    return true;
}

// ------------------------------------------------------------- the kernel
struct KArgs {
    const double2* pos_s;
    const int32_t* perm;
    const int32_t* start;
    MeshD m;
    Grid g;
    int64_t n_nodes;
    BuildOut out;
    int hw0, levels;
    unsigned long long* diag;
};

__device__ void write_node(const KArgs& a, int64_t node, const Support& S, int n, uint32_t meta,
                           const int32_t* perm) {
    const int64_t nn = a.n_nodes;
    for (int k = 0; k < n; ++k) {
        a.out.idx[k * nn + node] = perm[S.idx(k)];
        const double w = S.w[k * WG];
        a.out.w64[k * nn + node] = w;
        if (a.out.w32) a.out.w32[k * nn + node] = static_cast<float>(w);
        a.out.mem[k * nn + node] = static_cast<uint8_t>(S.bits(k));
    }
    a.out.meta[node] = meta;
}

__global__ void __launch_bounds__(WG) k_build(KArgs a) {
    __shared__ int32_t su[KMAX * WG];
    __shared__ double sw[KMAX * WG];
    const int tid = threadIdx.x;
    const int64_t node = static_cast<int64_t>(blockIdx.x) * WG + tid;
    if (node >= a.n_nodes) return;

    const int stride = a.m.nx + 1;
    const int i = static_cast<int>(node % stride);
    const int j = static_cast<int>(node / stride);
    const double2 q = make_double2(add_rn(a.m.x0, mul_rn(static_cast<double>(i), a.m.H)),
                                   add_rn(a.m.y0, mul_rn(static_cast<double>(j), a.m.H)));
    const bool ring = i == 0 || j == 0 || i == a.m.nx || j == a.m.ny;
    const int cbx = i * a.g.kb, cby = j * a.g.kb;

    Ctx c;
    c.pos = a.pos_s;
    c.perm = a.perm;
    c.start = a.start;
    c.g = a.g;
    c.neardeg = 0;
    Support S;
    S.u = su + tid;
    S.w = sw + tid;
    S.n = 0;

    uint32_t type = ring ? NT_RING : NT_INTERIOR;
    uint32_t flags = 0;
    int T[3] = {0, 0, 0};
    int st = R_FAIL;
    const int big = max(a.g.nbx, a.g.nby) + 1;

    if (!ring) {
        for (int level = 0;; ++level) {
            const int hw = level < a.levels ? (a.hw0 << level) : big;
            c.R = make_region(a.g, cbx, cby, hw);
            S.n = 0;
            st = locate(c, q, T);
            if (st == R_OK) st = ring_into(c, T, 0, S);
            if (st == R_OK) st = ring_into(c, T, 1, S);
            if (st == R_OK) st = ring_into(c, T, 2, S);
            if (st != R_MORE) break;
            if (c.R.global) {
                st = R_FAIL;
                break;
            }
            flags |= MF_ESCALATED;
        }
        if (c.R.global) flags |= MF_GLOBAL;
        if (st == R_OUTSIDE) type = NT_OUTSIDE;
        else if (st == R_CAP) {
            type = NT_FAILED;
            atomicAdd(&a.diag[D_CAP], 1ull);
        } else if (st != R_OK) type = NT_FAILED;
    }

    // every vertex of T lies in the others' rings; guard the LDS indexing anyway
    if (type == NT_INTERIOR && (S.find(T[0]) < 0 || S.find(T[1]) < 0 || S.find(T[2]) < 0)) type = NT_FAILED;
    if (type == NT_INTERIOR) {
        const int n = S.n;
        const int lt[3] = {S.find(T[0]), S.find(T[1]), S.find(T[2])};
        const double2 P0 = c.pos[T[0]], P1 = c.pos[T[1]], P2 = c.pos[T[2]];
        // barycentric coordinates of q in T (linear FE, eqs. C0, C1)
        const double D = orient(P0, P1, P2);
        const double phi[3] = {orient(q, P1, P2) / D, orient(P0, q, P2) / D, orient(P0, P1, q) / D};
        for (int k = 0; k < n; ++k) S.w[k * WG] = 0.0;
        for (int k = 0; k < 3; ++k) S.w[lt[k] * WG] += phi[k];
        for (int e = 0; e < 3; ++e) {
            const int pa = e, pb = (e + 1) % 3;
            const double2 rn = c.pos[T[pa]], rs = c.pos[T[pb]];
            const double cxm = 0.5 * (rn.x + rs.x), cym = 0.5 * (rn.y + rs.y);
            const double dxv = rn.x - rs.x, dyv = rn.y - rs.y;
            const double is = 1.0 / sqrt(dxv * dxv + dyv * dyv);
            const int mask = (1 << pa) | (1 << pb);
            auto member = [&](int k) { return (S.bits(k) & mask) != 0; };
            auto coord = [&](int k, double& x, double& y) {
                const double2 p = c.pos[S.idx(k)];
                x = (p.x - cxm) * is;
                y = (p.y - cym) * is;
            };
            Moments mo;
            mo.zero();
            for (int k = 0; k < n; ++k) {
                if (!member(k)) continue;
                double x, y;
                coord(k, x, y);
                mo.add(x, y);
            }
            const double dx = dxv * is, dy = dyv * is;
            const double b[6] = {0.0, 0.0, 0.0, -0.5 * dx * dx, -0.5 * dx * dy, -0.5 * dy * dy};
            double y[6];
            if (!min_norm(mo, b, n, member, coord, y)) {
                flags |= MF_RANKDEF;
                atomicAdd(&a.diag[D_RANKDEF], 1ull);
            }
            const double coef = 2.0 * phi[pa] * phi[pb];
            for (int k = 0; k < n; ++k) {
                if (!member(k)) continue;
                double x, yy;
                coord(k, x, yy);
                double p[6];
                monos(x, yy, p);
                const double A = p[0] * y[0] + p[1] * y[1] + p[2] * y[2] + p[3] * y[3] + p[4] * y[4] + p[5] * y[5];
                S.w[k * WG] += coef * A;
            }
        }
        if (c.neardeg) flags |= MF_NEARDEG;
        write_node(a, node, S, n, meta_pack(NT_INTERIOR, n, lt[0], lt[1], lt[2], flags), a.perm);
    } else if (type == NT_RING || type == NT_OUTSIDE) {
        // closure: K nearest particles (ties by user id), minimum-norm
        // quadratic moment weights.
        int nn[KNN];
        double dd[KNN];
        int uu[KNN];
        int kk = 0;
        for (int level = 0;; ++level) {
            const int hw = level < a.levels ? (a.hw0 << level) : big;
            c.R = make_region(a.g, cbx, cby, hw);
#pragma unroll
            for (int s = 0; s < KNN; ++s) {
                nn[s] = -1;
                dd[s] = INFINITY;
                uu[s] = INT_MAX;
            }
            kk = 0;
            for (int by = c.R.by0; by < c.R.by1; ++by) {
                const int row = by * c.g.nbx;
                const int s0 = c.start[row + c.R.bx0], e0 = c.start[row + c.R.bx1];
                for (int t = s0; t < e0; ++t) {
                    const double2 p = c.pos[t];
                    const double dx = p.x - q.x, dy = p.y - q.y;
                    const double d2 = dx * dx + dy * dy;
                    if (d2 > dd[KNN - 1]) continue;
                    const int u = c.perm[t];
                    if (d2 == dd[KNN - 1] && u >= uu[KNN - 1]) continue;
                    ++kk;
                    nn[KNN - 1] = t;
                    dd[KNN - 1] = d2;
                    uu[KNN - 1] = u;
#pragma unroll
                    for (int s = KNN - 1; s > 0; --s) {
                        const bool less = dd[s] < dd[s - 1] || (dd[s] == dd[s - 1] && uu[s] < uu[s - 1]);
                        if (less) {
                            const int tn = nn[s];
                            nn[s] = nn[s - 1];
                            nn[s - 1] = tn;
                            const double td = dd[s];
                            dd[s] = dd[s - 1];
                            dd[s - 1] = td;
                            const int tu = uu[s];
                            uu[s] = uu[s - 1];
                            uu[s - 1] = tu;
                        }
                    }
                }
            }
            if (c.R.global) break;
            if (kk >= KNN && disk_inside(c.R, q.x, q.y, sqrt(dd[KNN - 1]))) break;
            flags |= MF_ESCALATED;
        }
        if (c.R.global) flags |= MF_GLOBAL;
        const int n = kk < KNN ? kk : KNN;
        S.n = 0;
        for (int s = 0; s < n; ++s) S.u[s * WG] = nn[s];
        S.n = n;
        if (n == 0) {
            type = NT_FAILED;
        } else {
            // centroid and RMS radius: any centre and scale give the same
            // weights; these keep the moment matrix well conditioned.
            double mx = 0.0, my = 0.0;
            for (int s = 0; s < n; ++s) {
                const double2 p = c.pos[nn[s]];
                mx += p.x;
                my += p.y;
            }
            mx /= n;
            my /= n;
            double r2 = 0.0;
            for (int s = 0; s < n; ++s) {
                const double2 p = c.pos[nn[s]];
                r2 += (p.x - mx) * (p.x - mx) + (p.y - my) * (p.y - my);
            }
            const double isc = r2 > 0.0 ? 1.0 / sqrt(r2 / n) : 1.0;
            auto member = [&](int) { return true; };
            auto coord = [&](int k, double& x, double& y) {
                const double2 p = c.pos[S.idx(k)];
                x = (p.x - mx) * isc;
                y = (p.y - my) * isc;
            };
            Moments mo;
            mo.zero();
            for (int k = 0; k < n; ++k) {
                double x, y;
                coord(k, x, y);
                mo.add(x, y);
            }
            double b[6];
            monos((q.x - mx) * isc, (q.y - my) * isc, b);
            double y[6];
            if (!min_norm(mo, b, n, member, coord, y)) {
                flags |= MF_RANKDEF;
                atomicAdd(&a.diag[D_RANKDEF], 1ull);
            }
            for (int k = 0; k < n; ++k) {
                double x, yy;
                coord(k, x, yy);
                double p[6];
                monos(x, yy, p);
                S.w[k * WG] = p[0] * y[0] + p[1] * y[1] + p[2] * y[2] + p[3] * y[3] + p[4] * y[4] + p[5] * y[5];
            }
            if (c.neardeg) flags |= MF_NEARDEG;
            write_node(a, node, S, n, meta_pack(type, n, 0, 0, 0, flags), a.perm);
        }
    }
    if (type == NT_FAILED) {
        a.out.meta[node] = meta_pack(NT_FAILED, 0, 0, 0, 0, flags);
        atomicAdd(&a.diag[D_FAILED], 1ull);
    }

    // diagnostics: one atomic per wave for the common counters
    const unsigned long long interior = __ballot(type == NT_INTERIOR);
    const unsigned long long clos = __ballot(type == NT_RING || type == NT_OUTSIDE);
    const unsigned long long outside = __ballot(type == NT_OUTSIDE);
    const unsigned long long esc = __ballot((flags & MF_ESCALATED) != 0);
    const unsigned long long glob = __ballot((flags & MF_GLOBAL) != 0);
    int sup = (type == NT_FAILED) ? 0 : S.n;
    for (int off = 32; off > 0; off >>= 1) sup = max(sup, __shfl_xor(sup, off));
    int nd = c.neardeg;
    for (int off = 32; off > 0; off >>= 1) nd += __shfl_xor(nd, off);
    const int lane = __lane_id();
    const unsigned long long active = __ballot(true);
    if (lane == __ffsll(static_cast<long long>(active)) - 1) {
        if (interior) atomicAdd(&a.diag[D_INTERIOR], static_cast<unsigned long long>(__popcll(interior)));
        if (clos) atomicAdd(&a.diag[D_CLOSURE], static_cast<unsigned long long>(__popcll(clos)));
        if (outside) atomicAdd(&a.diag[D_OUTSIDE], static_cast<unsigned long long>(__popcll(outside)));
        if (esc) atomicAdd(&a.diag[D_ESCALATED], static_cast<unsigned long long>(__popcll(esc)));
        if (glob) atomicAdd(&a.diag[D_GLOBAL], static_cast<unsigned long long>(__popcll(glob)));
        if (nd) atomicAdd(&a.diag[D_NEARDEG], static_cast<unsigned long long>(nd));
        atomicMax(&a.diag[D_SUPMAX], static_cast<unsigned long long>(sup));
    }
}

}  // namespace

int build_weights(const BinBuffers& b, const MeshD& m, const Grid& g, int64_t N, const BuildOut& out,
                  const BuildParams& prm, unsigned long long* diag, hipStream_t st) {
    PhaseTimer _timer(PH_BUILD, st);
    (void)N;
    KArgs a;
    a.pos_s = reinterpret_cast<const double2*>(b.pos_s);
    a.perm = b.perm;
    a.start = b.start;
    a.m = m;
    a.g = g;
    a.n_nodes = static_cast<int64_t>(m.nx + 1) * (m.ny + 1);
    a.out = out;
    a.hw0 = prm.hw0;
    a.levels = prm.levels;
    a.diag = diag;
    const int blocks = static_cast<int>((a.n_nodes + WG - 1) / WG);
    k_build<<<blocks, WG, 0, st>>>(a);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
