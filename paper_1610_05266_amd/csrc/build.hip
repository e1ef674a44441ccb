// Weight build: psi_mu(r_i) at every mesh node (App. B of the paper).
//
// For an interior node q:
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
// circumdisk lies inside a region all of whose particles were candidates.
// Near-ties of the FP64 predicates (|det| within a forward error bound) are
// counted and broken by the user particle id.
//
// Execution: the FAST kernel stages each 8 x 8-node tile's bin region in LDS
// and gives each node a quad of four lanes holding the particles within a
// radius Rf of the node as 16-bit indices into that region, dealt in turn
// over the lanes, so each gift-wrapping step is a short loop over LDS
// positions plus a two-step quad reduction; a decision is certified when its
// disk lies in the disk of radius Rf around the node (boundary-ring nodes
// take their K nearest particles, certified the same way).  A node that
// cannot be certified there is appended to a list for the SLOW kernel on a
// side stream: three waves per node, each running the same wedge and walk
// and then the ring of one vertex, over square bin regions that double in
// size up to all particles; the first wave merges the rings and weights the
// row.  Meanwhile the WEIGHTS kernel (a quad per node) turns every row of the
// fast pass into weights.  Both passes produce the same rows in the same
// order and use the same weighting code, so the result of a node does not
// depend on the pass that found its triangle.  With the linear option the
// search stops at T and the row is phi alone.  With the periodic option
// the box is a torus: the exact path's regions wrap across its sides and read
// every particle at its image nearest to the node, the fast pass keeps the
// nodes whose windows stay inside the box, there are no closure nodes, and
// the seam nodes' rows are copies of the first column and row.  The end of
// the file builds the mesh-side counterpart: the coefficient table of every
// mesh edge.
#include <algorithm>
#include <cfloat>
#include <climits>

#include "algebra.h"
#include "kernels.h"

namespace p2m {

namespace {

constexpr double EPS = DBL_EPSILON;
constexpr int WAVE = 64;
constexpr int SWG = 192;       // slow kernel: three waves per node, one per ring
constexpr int QL = 4;          // lanes per node in the quad kernels
constexpr int NS_MAX = 10;     // candidate slots per lane (fast kernel), at most
constexpr int QWG = 256;       // quad kernels: 64 nodes per block
constexpr int QPB = QWG / QL;
constexpr int KPITCH = KMAX + 1;  // LDS row pitch of per-quad support lists
constexpr uint32_t IDX_MASK = 0x0fffffffu;

enum Result : int { R_OK = 0, R_MORE = 1, R_OUTSIDE = 2, R_FAIL = 3, R_CAP = 4 };

__device__ __forceinline__ double orient(double2 p, double2 q, double2 r) {
    return (q.x - p.x) * (r.y - p.y) - (q.y - p.y) * (r.x - p.x);
}

// ------------------------------------------------- candidate comparisons
// Bisector key of candidate b for the edge v -> a on side sgn: the circumcentre
// of (v, a, b) is v + A/2 + (num / 2cr) sgn perp(A), with A = a - v, B = b - v,
// num = B.(B - A), cr = sgn cross(A, B) > 0.  Smaller key = touched first.
struct Key {
    int t;           // sorted index, -1 = none
    double num, cr;  // key = num / cr
    double Nm, Cm;   // magnitudes for the forward error bound
    double bx, by;   // the candidate's position
};

__device__ __forceinline__ Key no_key() {
    Key k;
    k.t = -1;
    k.num = k.cr = k.Nm = k.Cm = k.bx = k.by = 0.0;
    return k;
}

__device__ __forceinline__ Key key_of(int t, double2 v, double2 a, double2 b, double sgn, int& neardeg) {
    Key k;
    const double Ax = a.x - v.x, Ay = a.y - v.y;
    const double Bx = b.x - v.x, By = b.y - v.y;
    k.cr = sgn * (Ax * By - Ay * Bx);
    k.Cm = fabs(Ax) * fabs(By) + fabs(Ay) * fabs(Bx);
    k.num = Bx * (Bx - Ax) + By * (By - Ay);
    k.Nm = Bx * Bx + By * By + fabs(Bx * Ax) + fabs(By * Ay);
    k.bx = b.x;
    k.by = b.y;
    k.t = t;
    if (k.cr <= 4.0 * EPS * k.Cm) {
        if (k.cr > -4.0 * EPS * k.Cm) ++neardeg;  // (nearly) on the line through v, a
        k.t = -1;
    }
    return k;
}

// true if `o` is touched before `m` (ties within the error bound go to the
// smaller user id; `uid` maps a sorted index to the user id).
template <class Uid>
__device__ __forceinline__ bool key_better(const Key& o, const Key& m, Uid uid, int& neardeg) {
    if (o.t < 0) return false;
    if (m.t < 0) return true;
    if (o.t == m.t) return false;
    const double lhs = o.num * m.cr, rhs = m.num * o.cr;
    const double err = 16.0 * EPS * (o.Nm * m.Cm + m.Nm * o.Cm);
    if (lhs < rhs - err) return true;
    if (lhs > rhs + err) return false;
    ++neardeg;
    return uid(o.t) < uid(m.t);
}

// With FAST the division and the square root are the hardware's reciprocal
// and reciprocal square root, each refined by two Newton steps (a few ulp:
// the certificates that use the circle leave margins of 1e-9 r and 1e-12 Rf),
// and a divisor or squared radius outside [2^-900, 2^900] (or not a number)
// gives an infinite radius, which no certificate accepts: the node is then
// left to the exact path, which uses the correctly rounded forms.
template <bool FAST>
__device__ __forceinline__ void circumcircle(const Key& k, double2 v, double2 a, double sgn, double& cx,
                                             double& cy, double& rr) {
    const double Ax = a.x - v.x, Ay = a.y - v.y;
    if constexpr (FAST) {
        const double d = 2.0 * k.cr;
        double y = __builtin_amdgcn_rcp(d);
        y = fma(fma(-d, y, 1.0), y, y);
        y = fma(fma(-d, y, 1.0), y, y);
        const double tk = k.num * y;
        const double ox = 0.5 * Ax - sgn * tk * Ay;
        const double oy = 0.5 * Ay + sgn * tk * Ax;
        cx = v.x + ox;
        cy = v.y + oy;
        const double x = ox * ox + oy * oy;
        // g -> sqrt(x), h -> 1 / (2 sqrt(x)): one coupled step, one residual step
        const double r0 = __builtin_amdgcn_rsq(x);
        double g = x * r0, h = 0.5 * r0;
        const double e = fma(-g, h, 0.5);
        g = fma(g, e, g);
        h = fma(h, e, h);
        g = fma(fma(-g, g, x), h, g);
        const bool ok = (d >= 0x1p-900) & (d <= 0x1p900) & (x >= 0x1p-900) & (x <= 0x1p900);
        rr = ok ? g : INFINITY;
    } else {
        const double tk = k.num / (2.0 * k.cr);
        const double ox = 0.5 * Ax - sgn * tk * Ay;
        const double oy = 0.5 * Ay + sgn * tk * Ax;
        cx = v.x + ox;
        cy = v.y + oy;
        rr = sqrt(ox * ox + oy * oy);
    }
}

// Butterfly reductions over groups of W lanes: every lane of a group ends
// with the same answer.  Near-ties met during the reduction are counted once
// per pair (by its lower lane).
template <int W, class Uid>
__device__ __forceinline__ void reduce_key(Key& best, Uid uid, int lane, int& nd) {
#pragma unroll
    for (int m = 1; m < W; m <<= 1) {
        Key o;
        o.t = lane_xor<W>(best.t, m);
        o.num = lane_xor<W>(best.num, m);
        o.cr = lane_xor<W>(best.cr, m);
        o.Nm = lane_xor<W>(best.Nm, m);
        o.Cm = lane_xor<W>(best.Cm, m);
        o.bx = lane_xor<W>(best.bx, m);
        o.by = lane_xor<W>(best.by, m);
        int dummy = 0;
        if (key_better(o, best, uid, (lane & m) ? dummy : nd)) best = o;
    }
}

template <int W, class Uid>
__device__ __forceinline__ void reduce_nearest(double& d2, int& t, double2& p, Uid uid) {
#pragma unroll
    for (int m = 1; m < W; m <<= 1) {
        const double od = lane_xor<W>(d2, m);
        const int ot = lane_xor<W>(t, m);
        const double ox = lane_xor<W>(p.x, m), oy = lane_xor<W>(p.y, m);
        bool take = false;
        if (ot >= 0 && ot != t) {
            if (t < 0 || od < d2) take = true;
            else if (od == d2) take = uid(ot) < uid(t);
        }
        if (take) {
            d2 = od;
            t = ot;
            p = make_double2(ox, oy);
        }
    }
}

// ---- whole-wave selections by ballot -------------------------------------
// A wave-wide argmin needs the butterfly only to agree on a value: the
// minimum of one double is found first, the lanes that might tie it are
// singled out by a ballot, and the winner is read from its lane.  The full
// exact butterfly runs only when a near-tie is possible.
__device__ __forceinline__ int read_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// Value of v in the mirrored lane of the same 16-lane row (DPP, no LDS round
// trip): CTRL 0x141 mirrors each half row (lane i <-> 7 - i), 0x140 the
// whole row (i <-> 15 - i).
template <int CTRL>
__device__ __forceinline__ double row_mirror(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// Minimum over the wave, in every lane (every lane active).  Within a row of
// 16 lanes each exchange merges two disjoint groups (quad permutes, then the
// half-row and row mirrors); the four row minima are then read as scalars.
__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, lane_xor<4>(v, 1));
    v = fmin(v, lane_xor<4>(v, 2));
    v = fmin(v, row_mirror<0x141>(v));
    v = fmin(v, row_mirror<0x140>(v));
    return fmin(fmin(read_lane(v, 0), read_lane(v, 16)), fmin(read_lane(v, 32), read_lane(v, 48)));
}
__device__ __forceinline__ Key read_key(const Key& k, int l) {
    Key o;
    o.t = read_lane(k.t, l);
    o.num = read_lane(k.num, l);
    o.cr = read_lane(k.cr, l);
    o.Nm = read_lane(k.Nm, l);
    o.Cm = read_lane(k.Cm, l);
    o.bx = read_lane(k.bx, l);
    o.by = read_lane(k.by, l);
    return o;
}

// Exact wave argmin of bisector keys (key_better order).  The lane whose
// rounded quotient num/cr is smallest is the answer unless some other lane's
// key is within the forward error bound of it (or below): then, and only
// then, the exact butterfly decides (and counts the near-ties).
template <class Uid>
__device__ __forceinline__ void wave_best_key(Key& best, Uid uid, int lane, int& nd) {
    const double kv = best.t >= 0 ? best.num / best.cr : INFINITY;
    const double km = wave_min(kv);
    if (km == INFINITY) {
        best = no_key();
        return;
    }
    const int ml = __ffsll(static_cast<long long>(__ballot(kv == km))) - 1;
    const Key m = read_key(best, ml);
    bool cont = false;
    if (best.t >= 0 && best.t != m.t) {
        const double lhs = best.num * m.cr, rhs = m.num * best.cr;
        const double err = 16.0 * EPS * (best.Nm * m.Cm + m.Nm * best.Cm);
        cont = !(lhs > rhs + err);
    }
    if (__ballot(cont) == 0) {
        best = m;
        return;
    }
    reduce_key<WAVE>(best, uid, lane, nd);
    // every lane holds the answer; read as a scalar it is visibly
    // wave-uniform, so the branches that depend on it stay scalar
    best = read_key(best, 0);
}

// Wave argmin of squared distances, ties by user id.
__device__ __forceinline__ void wave_nearest(double& d2, int& t, double2& p, const int32_t* perm) {
    const double v = t >= 0 ? d2 : INFINITY;
    const double mv = wave_min(v);
    const unsigned long long tied = __ballot(t >= 0 && v == mv);
    if (tied == 0) {
        t = -1;
        d2 = INFINITY;
        p = make_double2(0.0, 0.0);
        return;
    }
    if (__popcll(tied) == 1) {
        const int l = __ffsll(static_cast<long long>(tied)) - 1;
        t = read_lane(t, l);
        d2 = read_lane(d2, l);
        p = make_double2(read_lane(p.x, l), read_lane(p.y, l));
        return;
    }
    reduce_nearest<WAVE>(d2, t, p, [&](int u) { return perm[u]; });
    t = read_lane(t, 0);
    d2 = read_lane(d2, 0);
    p = make_double2(read_lane(p.x, 0), read_lane(p.y, 0));
}

template <int W>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = 1; m < W; m <<= 1) v += lane_xor<W>(v, m);
    return v;
}

// ------------------------------------------------ slow candidate source
struct Region {
    // bins [bx0, bx1) x [by0, by1); in a periodic box unwrapped (they may
    // pass the box sides), each bin row then read as nseg runs of columns
    int bx0, bx1, by0, by1;
    int nseg;
    double xlo, xhi, ylo, yhi;
    bool global;

    __device__ int nrun() const { return (by1 - by0) * nseg; }
    // run v: key of its bin row's first bin and its columns [c0, c1)
    __device__ void run(const Grid& g, int v, int& base, int& c0, int& c1) const {
        int by = by0 + (nseg == 1 ? v : v >> 1);
        by += by < 0 ? g.nby : (by >= g.nby ? -g.nby : 0);
        base = by * g.nbx;
        c0 = bx0;
        c1 = bx1;
        if (nseg == 2) {
            const bool first = (v & 1) == 0;
            if (bx0 < 0) {
                c0 = first ? bx0 + g.nbx : 0;
                c1 = first ? g.nbx : bx1;
            } else {
                c0 = first ? bx0 : 0;
                c1 = first ? g.nbx : bx1 - g.nbx;
            }
        }
    }
};

// Periodic region: half-width hw bins around the node's bin corner, kept one
// bin inside the half-period on every side so that the particles read in it
// are the images nearest to the node; wider, every particle at its nearest
// image, certified inside that largest window.
__device__ Region make_region_periodic(const Grid& g, int cbx, int cby, int hw) {
    Region R;
    const double m = 1e-9 * g.bw;
    const int hx = (g.nbx - 2) / 2, hy = (g.nby - 2) / 2;
    R.global = hw > hx || hw > hy;
    const int wx = R.global ? hx : hw, wy = R.global ? hy : hw;
    R.xlo = g.x0 + (cbx - wx) * g.bw + m;
    R.xhi = g.x0 + (cbx + wx) * g.bw - m;
    R.ylo = g.y0 + (cby - wy) * g.bw + m;
    R.yhi = g.y0 + (cby + wy) * g.bw - m;
    if (R.global) {
        R.bx0 = 0;
        R.bx1 = g.nbx;
        R.by0 = 0;
        R.by1 = g.nby;
    } else {
        R.bx0 = cbx - hw;
        R.bx1 = cbx + hw;
        R.by0 = cby - hw;
        R.by1 = cby + hw;
    }
    R.nseg = (R.bx0 < 0 || R.bx1 > g.nbx) ? 2 : 1;
    return R;
}

__device__ Region make_region(const Grid& g, int cbx, int cby, int hw) {
    Region R;
    R.nseg = 1;
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

// A whole wave per node, scanning a square region of bins (sides on the
// mesh boundary are walls: no particle lies beyond them).  The region's
// particles are staged once per region in LDS when they fit (STAGE entries
// per wave), else streamed from the sorted arrays on every scan; either way
// they are dealt round-robin over the 64 lanes.
constexpr int STAGE = 512;

// REGS: regions of at most 2 WAVE particles (and WAVE bin rows) held in
// registers instead of LDS (fewer LDS reads per query, more registers).
template <bool PER, bool REGS = true>
struct WaveSource {
    static constexpr bool kFastCircle = false;
    // (every member inlined: a call would put the source in scratch memory)
    static constexpr bool per = PER;
    const double2* __restrict__ pos;
    const int32_t* __restrict__ perm;
    const int32_t* __restrict__ start;
    Grid g;
    Region R;
    MeshD m;
    double2 q;     // the node (periodic box: positions are its nearest images)
    int neardeg;
    int ring_mark;
    int lane;
    double2* lp;   // LDS stage of this wave [STAGE]
    int32_t* lt;   // sorted indices of the staged particles
    int ln;        // staged count, -1 when streaming
    // (REGS) regions held in registers: flat element f by lane f % WAVE, as
    // the staged loop deals them
    int nreg;      // particles held in registers, -1 when not
    double2 rp0, rp1;
    int rt0, rt1;

    // every particle was a candidate (a periodic box has no hull: its widest
    // window answers only what it certifies)
    __device__ __forceinline__ bool global() const { return R.global && !per; }
    // near-tie count when the rings phase begins
    __device__ __forceinline__ void mark_rings() { ring_mark = neardeg; }
    __device__ __forceinline__ void progress(int) const {}
    __device__ __forceinline__ double2 at(int t) const {
        const double2 p = pos[t];
        return per ? image_near(m, p, q) : p;
    }
    __device__ __forceinline__ double2 P(int t) const { return at(t); }
    __device__ __forceinline__ bool certify(double cx, double cy, double r) const {
        r *= 1.0 + 1e-9;
        return cx - r >= R.xlo && cx + r <= R.xhi && cy - r >= R.ylo && cy + r <= R.yhi;
    }
    __device__ __forceinline__ void set_region(const Region& reg) {
        R = reg;
        // run lengths, one lane per run (a bin row, or a part of one that
        // wraps), 64 runs at a time
        const int nrow = R.nrun();
        int total = 0, rs = 0, rpre = 0;  // this lane's run (first 64 runs): start, flat offset
        for (int r0 = 0; r0 < nrow; r0 += WAVE) {
            const int r = r0 + lane;
            int len = 0, s0 = 0;
            if (r < nrow) {
                int row, c0, c1;
                R.run(g, r, row, c0, c1);
                s0 = start[row + c0];
                len = start[row + c1] - s0;
            }
            int inc = len;
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                const int o = __shfl_up(inc, d);
                if (lane >= d) inc += o;
            }
            if (r0 == 0) {
                rs = s0;
                rpre = inc - len;
            }
            total += read_lane(inc, WAVE - 1);
        }
        nreg = -1;
        if constexpr (REGS) {
            if (total <= 2 * WAVE && nrow <= WAVE) {
                // each lane finds the rows of its flat elements lane and lane + WAVE
                int t0 = -1, t1 = -1;
                for (int r = 0; r < nrow; ++r) {
                    const int sr = read_lane(rs, r), pr = read_lane(rpre, r);
                    const int pe = r + 1 < nrow ? read_lane(rpre, r + 1) : total;
                    if (lane >= pr && lane < pe) t0 = sr + lane - pr;
                    if (lane + WAVE >= pr && lane + WAVE < pe) t1 = sr + lane + WAVE - pr;
                }
                rt0 = t0;
                rt1 = t1;
                rp0 = at(t0 >= 0 ? t0 : 0);
                rp1 = at(t1 >= 0 ? t1 : 0);
                nreg = total;
                ln = -1;
                return;
            }
        }
        ln = total <= STAGE ? total : -1;
        if (ln < 0) return;
        int flat = 0;
        for (int v = 0; v < nrow; ++v) {
            int row, c0, c1;
            R.run(g, v, row, c0, c1);
            const int s = start[row + c0], e = start[row + c1];
            for (int t = s + lane; t < e; t += WAVE) {
                lp[flat + t - s] = at(t);
                lt[flat + t - s] = t;
            }
            flat += e - s;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    template <class F>
    __device__ __forceinline__ void scan(F&& f) const {
        if constexpr (REGS) {
            if (nreg >= 0) {
                if (lane < nreg) f(rt0, rp0);
                if (lane + WAVE < nreg) f(rt1, rp1);
                return;
            }
        }
        if (ln >= 0) {
            for (int k = lane; k < ln; k += WAVE) f(lt[k], lp[k]);
            return;
        }
        int flat = 0;
        for (int v = 0, nv = R.nrun(); v < nv; ++v) {
            int row, c0, c1;
            R.run(g, v, row, c0, c1);
            const int s = start[row + c0], e = start[row + c1];
            for (int t = s + ((lane - flat) & (WAVE - 1)); t < e; t += WAVE) f(t, at(t));
            flat += e - s;
        }
    }
    __device__ __forceinline__ int nearest(double2 c, int exclude, double& d2best, double2& pbest) {
        int best = -1;
        d2best = INFINITY;
        pbest = make_double2(0.0, 0.0);
        scan([&](int t, double2 p) {
            if (t == exclude) return;
            const double dx = p.x - c.x, dy = p.y - c.y;
            const double d2 = dx * dx + dy * dy;
            if (d2 < d2best || (d2 == d2best && best >= 0 && perm[t] < perm[best])) {
                best = t;
                d2best = d2;
                pbest = p;
            }
        });
        wave_nearest(d2best, best, pbest, perm);
        return best;
    }
    __device__ __forceinline__ Key wrap(int iv, double2 v, int ia, double2 a, double sgn) {
        Key best = no_key();
        auto uid = [&](int t) { return perm[t]; };
        int nd = 0;
        scan([&](int t, double2 b) {
            if (t == iv || t == ia) return;
            const Key k = key_of(t, v, a, b, sgn, nd);
            if (key_better(k, best, uid, nd)) best = k;
        });
        wave_best_key(best, uid, lane, nd);
        neardeg += nd;
        return best;
    }
};

// -------------------------------------------------- fast candidate source
// Four lanes of a quad hold the node's candidates (particles within Rf of
// the node q); every query is a lane-local loop plus a two-step reduction,
// after which all four lanes agree on the answer.  The candidates are
// 16-bit indices into the tile's region staged in LDS (two per register),
// positions are read from there: the registers they free let four blocks
// share a CU.  Indices t of this source are staged indices; sorted(t) is the
// particle's index in the sorted arrays.
template <int NS>
struct QuadSource {
    static constexpr bool kFastCircle = true;
    const int32_t* __restrict__ perm;
    const double2* lpos;  // the staged positions
    const int32_t* lrb;   // staged index of the first particle of each staged row (nrow + 1)
    const int32_t* lrs;   // sorted index of the first particle of each staged row
    int nrow;
    double2 q;
    double Rf;
    uint32_t ci_[(NS + 1) / 2];  // candidate s in bits 16 (s & 1) .. of word s / 2
    // some lane of the wave that runs the Delaunay routine holds NS
    // candidates (wave-uniform); else every query skips the last slot, which
    // all those lanes leave empty
    bool use_last = true;
    int n;
    int lane;  // 0..3

    __device__ int cand(int s) const { return static_cast<int>((ci_[s >> 1] >> ((s & 1) << 4)) & 0xFFFFu); }
    __device__ int sorted(int t) const {
        int lo = 0, hi = nrow - 1;  // the staged row holding t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lrb[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        return lrs[lo] + (t - lrb[lo]);
    }
    __device__ int uid(int t) const { return perm[sorted(t)]; }
    __device__ bool global() const { return false; }
    // the disk (c, r) inside the disk (q, Rf), with margins far above the
    // rounding of either side: |c - q| + r (1 + 1e-9) <= Rf (1 - 1e-12),
    // compared squared (one square root fewer per step)
    __device__ bool certify(double cx, double cy, double r) const {
        const double dx = cx - q.x, dy = cy - q.y;
        const double u = Rf * (1.0 - 1e-12) - r * (1.0 + 1e-9);
        return u >= 0.0 && dx * dx + dy * dy <= u * u;
    }
    __device__ int nearest(double2 c, int exclude, double& d2best, double2& pbest) {
        int best = -1;
        d2best = INFINITY;
        pbest = make_double2(0.0, 0.0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s == NS - 1 && !use_last) break;
            if (s >= n) continue;
            const int t = cand(s);
            if (t == exclude) continue;
            const double2 b = lpos[t];
            const double dx = b.x - c.x, dy = b.y - c.y;
            const double d2 = dx * dx + dy * dy;
            if (d2 < d2best || (d2 == d2best && best >= 0 && uid(t) < uid(best))) {
                best = t;
                d2best = d2;
                pbest = b;
            }
        }
        reduce_nearest<QL>(d2best, best, pbest, [&](int u) { return uid(u); });
        return best;
    }
    __device__ double2 P(int t) const { return lpos[t]; }
    __device__ void mark_rings() {}
    // Issue priority by progress through the rings (the iteration count is
    // wave-uniform): a CU holds four blocks that start together, and the
    // arbiter favours the oldest waves; lowering a wave's priority as it
    // advances lets the waves behind it catch up, so that the CU keeps all
    // its waves (and their latency hiding) until near the end instead of
    // finishing its last block alone.
    __device__ __forceinline__ void progress(int it) const {
        if (it == 4) __builtin_amdgcn_s_setprio(2);
        else if (it == 8) __builtin_amdgcn_s_setprio(1);
        else if (it == 12) __builtin_amdgcn_s_setprio(0);
    }
    // A branch-free loop that compares bisector keys against a static
    // forward error bound valid for every candidate (all candidates, and v
    // and a, lie within Rf of q, so |A|, |B| <= 2 Rf and both error
    // magnitudes of key_of are <= 8 Rf^2).  Outside that bound its decisions
    // are the exact ones.  When any comparison falls inside it -- a near
    // tie, or a candidate nearly on the line through v and a -- the answer
    // is t = -2 and the node is left to the wave path, which compares with
    // per-candidate bounds and breaks ties by user id.
    __device__ Key wrap(int iv, double2 v, int ia, double2 a, double sgn) {
        const double Ax = a.x - v.x, Ay = a.y - v.y;
        const double nx = -sgn * Ay, ny = sgn * Ax;  // sgn cross(A, B) = n . B
        const double R2 = Rf * Rf;
        const double crmin = 32.0 * EPS * R2;
        const double errS = 2048.0 * EPS * R2 * R2;
        // only the winner's index and key travel through the loop and the
        // quad reduction; its position is read back from LDS once at the end
        int bt = -1;
        double bn = 0.0, bc = 1.0;
        bool amb = false;
        if constexpr (NS <= 7) {
            // The key starts at a sentinel (num, cr) = (128 R^2, 0) that every
            // candidate on the left beats by more than the error bound
            // (0 - 128 R^2 cr < -128 R^2 crmin < -errS), so no test for "no
            // winner yet" is needed, and the tests are combined without
            // short circuits: the same decisions in fewer instructions (with
            // more slots the compiler keeps too many of them live)
            bn = 128.0 * R2;
            bc = 0.0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (s == NS - 1 && !use_last) break;
                const int t = cand(s);  // slots past n hold index 0
                const double2 b = lpos[t];
                const double Bx = b.x - v.x, By = b.y - v.y;
                const double cr = nx * Bx + ny * By;
                const double num = Bx * (Bx - Ax) + By * (By - Ay);
                const bool ok = (s < n) & (t != iv) & (t != ia);
                const bool left = ok & (cr > crmin);
                const double d = num * bc - bn * cr;
                amb |= (ok & (fabs(cr) <= crmin)) | (left & (fabs(d) <= errS));
                const bool take = left & (d < -errS);
                bt = take ? t : bt;
                bn = take ? num : bn;
                bc = take ? cr : bc;
                if (s & 1) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int m = 1; m < QL; m <<= 1) {
                const int ot = lane_xor<QL>(bt, m);
                const double on = lane_xor<QL>(bn, m), oc = lane_xor<QL>(bc, m);
                const double d = on * bc - bn * oc;
                const bool other = (ot >= 0) & (ot != bt);
                amb |= other & (fabs(d) <= errS);
                const bool take = other & (d < -errS);
                bt = take ? ot : bt;
                bn = take ? on : bn;
                bc = take ? oc : bc;
            }
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (s == NS - 1 && !use_last) break;
                const int t = cand(s);  // slots past n hold index 0
                const double2 b = lpos[t];
                const double Bx = b.x - v.x, By = b.y - v.y;
                const double cr = nx * Bx + ny * By;
                const double num = Bx * (Bx - Ax) + By * (By - Ay);
                const bool ok = s < n && t != iv && t != ia;
                const bool left = ok && cr > crmin;
                const double d = num * bc - bn * cr;
                amb = amb || (ok && fabs(cr) <= crmin) || (left && bt >= 0 && fabs(d) <= errS);
                const bool take = left && (bt < 0 || d < -errS);
                bt = take ? t : bt;
                bn = take ? num : bn;
                bc = take ? cr : bc;
                // at most two candidates' loads in flight: the registers of all
                // of them would cost the fourth wave per SIMD
                if (s & 1) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int m = 1; m < QL; m <<= 1) {
                const int ot = lane_xor<QL>(bt, m);
                const double on = lane_xor<QL>(bn, m), oc = lane_xor<QL>(bc, m);
                const double d = on * bc - bn * oc;
                const bool other = ot >= 0 && ot != bt;
                amb = amb || (other && bt >= 0 && fabs(d) <= errS);
                const bool take = other && (bt < 0 || d < -errS);
                bt = take ? ot : bt;
                bn = take ? on : bn;
                bc = take ? oc : bc;
            }
        }
        int am = amb ? 1 : 0;
        am |= lane_xor<QL>(am, 1);
        am |= lane_xor<QL>(am, 2);
        Key k;
        k.t = am ? -2 : bt;
        k.num = bn;
        k.cr = bc;
        k.Nm = k.Cm = 0.0;
        const double2 pb = lpos[bt >= 0 ? bt : 0];
        k.bx = pb.x;
        k.by = pb.y;
        return k;
    }
};

// ------------------------------------------------- the Delaunay routine
// Support list U of one node: sorted particle index | membership << 28,
// entry k at u[k].  The W lanes cooperating on a node search it together
// (lane l checks entries l, l + W, ...) and perform identical updates.
template <int W>
struct Support {
    int32_t* u;
    int n;
    int lane;
    __device__ int find(int t) const {
        int f = -1;
        for (int k = lane; k < n; k += W)
            if (static_cast<int>(static_cast<uint32_t>(u[k]) & IDX_MASK) == t) f = k;
        if constexpr (W == WAVE) {
            // entries are distinct: at most one lane found t
            const unsigned long long b = __ballot(f >= 0);
            return b ? read_lane(f, __ffsll(static_cast<long long>(b)) - 1) : -1;
        } else {
#pragma unroll
            for (int m = 1; m < W; m <<= 1) f = max(f, lane_xor<W>(f, m));
            return f;
        }
    }
    // Add t with membership bit `bit` (or the bit to its entry); returns
    // its position, or -1 when the list is full.
    __device__ __forceinline__ int add(int t, int bit) {
        const int f = find(t);
        int at = f;
        if (f >= 0) {
            const int e = u[f];
            __builtin_amdgcn_wave_barrier();
            u[f] = e | (bit << 28);
        } else {
            if (n >= KMAX) return -1;
            u[n] = t | (bit << 28);
            at = n++;
        }
        __builtin_amdgcn_wave_barrier();
        return at;
    }
    // The bit to the entry at position p (known to hold the particle).
    __device__ __forceinline__ void set_bit(int p, int bit) {
        const int e = u[p];
        __builtin_amdgcn_wave_barrier();
        u[p] = e | (bit << 28);
        __builtin_amdgcn_wave_barrier();
    }
};


// Support list of one node on the wave path, entry k in lane k (KROW <= 64):
// a search is one compare and a ballot, an insertion a select, with no LDS
// round trip.  Same entries and order as Support.
struct WaveSupport {
    int e;  // this lane's entry: sorted index | membership << 28 (lane < n)
    int n;
    int lane;
    __device__ int find(int t) const {
        const unsigned long long b =
            __ballot(lane < n && static_cast<int>(static_cast<uint32_t>(e) & IDX_MASK) == t);
        return b ? __ffsll(static_cast<long long>(b)) - 1 : -1;
    }
    // (updates as selects, not branches around stores: the struct then
    // stays in registers)
    __device__ __forceinline__ int add(int t, int bit) {
        const int f = find(t);
        if (f >= 0) {
            e |= lane == f ? bit << 28 : 0;
            return f;
        }
        if (n >= KROW) return -1;
        e = lane == n ? t | (bit << 28) : e;
        return n++;
    }
    __device__ __forceinline__ void set_bit(int p, int bit) { e |= lane == p ? bit << 28 : 0; }
    // Exchange the entries at positions a and b (wave-uniform).
    __device__ void swap(int a, int b) {
        const int ea = __builtin_amdgcn_readlane(e, a), eb = __builtin_amdgcn_readlane(e, b);
        if (lane == a) e = eb;
        if (lane == b) e = ea;
    }
};

// Positions in a support list of a triangle's three vertices, packed 7 bits
// each (position + 1; 0: not in the list), so that they stay in a register.
__device__ __forceinline__ int vertex_pos(int tpk, int k) {
    return static_cast<int>((static_cast<uint32_t>(tpk) >> (7 * k)) & 127u) - 1;
}
// Vertex k (particle t) into the list with membership bit `bit`: a bit set
// at its known position, else an add (and its position recorded).  False
// when the list is full.
template <class S_>
__device__ __forceinline__ bool add_vertex(S_& S, int& tpk, int k, int t, int bit) {
    const int p0 = vertex_pos(tpk, k);
    if (p0 >= 0) {
        S.set_bit(p0, bit);
        return true;
    }
    const int p = S.add(t, bit);
    if (p < 0) return false;
    tpk |= (p + 1) << (7 * k);
    return true;
}

// Delaunay work of one node q: the triangle T (CCW, sorted indices) of the
// particles' Delaunay triangulation that contains q, and the rings of its
// three vertices (into S, bit k for the ring of T[k]).  Three phases, each a
// loop around one gift-wrapping step:
//   wedge   rotate about the nearest particle n0 (from its nearest
//           neighbour a0, a Delaunay neighbour, on the side of q) to the
//           wedge holding q; the other way as well for a hull vertex (only a
//           global source sees one);
//   walk    visibility walk across the edge facing q;
//   rings   rotate about T[k] from the known triangle T back to it (clockwise
//           for the rest of an open fan of a hull vertex).
// Work is reused: when q lies in a triangle at n0, the ring of n0 only
// rotates over the part the wedge search did not visit (its apexes are kept
// in `vis`); the first step of rings 1 and 2 and the last step of ring 2 are
// triangles across an edge of T that an earlier ring already found.
// Returns R_OK, R_OUTSIDE (q outside the convex hull), R_MORE (not
// certified by this source), R_FAIL or R_CAP.
// With `only` == -2 the routine stops at the triangle: the list is T's three
// vertices (the linear FE functions need nothing else).
// With `only` in 0..2 the rings phase does just that ring: several waves
// can then run the three rings of one node side by side; the lists they
// return, merged in ring order, are this routine's list in the same order
// (ring k > 0 starting at T[k-1] meets first the apex that the previous
// ring saw last before T[k], where the chained version starts).
template <class G, class S_>
__device__ __forceinline__ int delaunay_node(G& g, double2 q, int Tout[3], S_& S, int32_t* vis, int only = -1, int vcap = KMAX) {
    // the current triangle as scalars, selected by value (an array indexed
    // at run time would live in scratch memory)
    int T0 = -1, T1 = -1, T2 = -1;
    auto tsel = [&](int i) { return i == 0 ? T0 : (i == 1 ? T1 : T2); };
    double d2;
    double2 v;
    const int n0 = g.nearest(q, -1, d2, v);
    if (n0 < 0) return R_MORE;
    if (!g.certify(q.x, q.y, sqrt(d2))) return R_MORE;
    double e2;
    double2 pa0;
    const int a0 = g.nearest(v, n0, e2, pa0);
    if (a0 < 0) return g.global() ? R_OUTSIDE : R_MORE;
    // the nearest neighbour of v is a Delaunay neighbour of v
    if (!g.certify(v.x, v.y, sqrt(e2))) return R_MORE;
    double cx, cy, rr;

    // ---- wedge: rotate about n0 from a0 towards q (counter-clockwise when
    // q lies left of or on the ray n0 -> a0, else clockwise) to the triangle
    // T = (n0, T1, T2) whose cone holds q: q left of or on n0 -> T1 and
    // strictly right of n0 -> T2.  The cones are half-open, so either
    // direction ends at the same triangle.  `vis` keeps a0 and the apexes
    // passed after it.
    double2 P0 = v, P1 = v, P2 = v;
    auto psel = [&](int i) { return i == 0 ? P0 : (i == 1 ? P1 : P2); };
    const double dir = orient(v, pa0, q) >= 0.0 ? 1.0 : -1.0;
    int cur = a0;
    double2 pcur = pa0;
    int nvis = 1;
    vis[0] = a0;
    bool found = false, open = false;
    for (int step = 0; step < 2 * KMAX; ++step) {
        const Key k = g.wrap(n0, v, cur, pcur, dir);
        if (k.t == -2) return R_MORE;
        if (k.t < 0) {
            if (!g.global()) return R_MORE;
            open = true;
            break;
        }
        circumcircle<G::kFastCircle>(k, v, pcur, dir, cx, cy, rr);
        if (!g.certify(cx, cy, rr)) return R_MORE;
        const double2 pk = make_double2(k.bx, k.by);
        // the triangle's two rays in counter-clockwise order
        const double2 plo = dir > 0.0 ? pcur : pk, phi = dir > 0.0 ? pk : pcur;
        if (d2 == 0.0 || (orient(v, plo, q) >= 0.0 && orient(v, phi, q) < 0.0)) {
            T0 = n0;
            T1 = dir > 0.0 ? cur : k.t;
            T2 = dir > 0.0 ? k.t : cur;
            P0 = v; P1 = plo; P2 = phi;
            found = true;
            break;
        }
        // a full turn (or a step past a0 through co-circular ties) without
        // finding the wedge: numerically inconsistent
        if (k.t == a0 || (orient(v, plo, pa0) > 0.0 && orient(v, pa0, phi) > 0.0)) return R_FAIL;
        if (nvis >= vcap) return R_CAP;
        vis[nvis++] = k.t;
        cur = k.t;
        pcur = pk;
    }
    if (!found && !open) return R_FAIL;
    if (!found) {
        // n0 is a hull vertex: rotate the other way from a0 over the rest of its fan
        nvis = 0;
        cur = a0;
        pcur = pa0;
        for (int step = 0; step < 2 * KMAX; ++step) {
            const Key k = g.wrap(n0, v, cur, pcur, -dir);
            if (k.t == -2) return R_MORE;
            if (k.t < 0) return d2 == 0.0 ? R_FAIL : R_OUTSIDE;  // q outside the open fan's cone
            const double2 pk = make_double2(k.bx, k.by);
            const double2 plo = dir > 0.0 ? pk : pcur, phi = dir > 0.0 ? pcur : pk;
            if (d2 == 0.0 || (orient(v, plo, q) >= 0.0 && orient(v, phi, q) < 0.0)) {
                T0 = n0;
                T1 = dir > 0.0 ? k.t : cur;
                T2 = dir > 0.0 ? cur : k.t;
                P0 = v; P1 = plo; P2 = phi;
                found = true;
                break;
            }
            if (k.t == a0) return R_FAIL;
            cur = k.t;
            pcur = pk;
        }
        if (!found) return R_FAIL;
    }

    // ---- walk towards q
    bool walked = false;
    for (int step = 0;; ++step) {
        int we;
        if (orient(P1, P2, q) < 0.0) we = 1;
        else if (orient(P2, P0, q) < 0.0) we = 2;
        else if (orient(P0, P1, q) < 0.0) we = 0;
        else break;
        if (step >= 256) return R_FAIL;
        // across edge X -> Y lies the triangle (Y, X, D), D left of Y -> X
        const int w1 = we == 2 ? 0 : we + 1;
        const int tX = tsel(we), tY = tsel(w1);
        const double2 qX = psel(we), qY = psel(w1);
        const Key k = g.wrap(tY, qY, tX, qX, 1.0);
        if (k.t == -2) return R_MORE;
        if (k.t < 0) return g.global() ? R_OUTSIDE : R_MORE;
        circumcircle<G::kFastCircle>(k, qY, qX, 1.0, cx, cy, rr);
        if (!g.certify(cx, cy, rr)) return R_MORE;
        T0 = tY; T1 = tX; T2 = k.t;
        P0 = qY; P1 = qX; P2 = make_double2(k.bx, k.by);
        walked = true;
    }

    // ---- the three rings
    // A counter-clockwise wedge search passed the ring of n0 from a0 to T1:
    // ring 0 rotates from T2 until it meets a0.  A clockwise one passed it
    // from T2 back to a0, which continues ring 0 counter-clockwise from T2.
    g.mark_rings();
    if (only == -2) {
        if (S.add(T0, 0) < 0 || S.add(T1, 0) < 0 || S.add(T2, 0) < 0) return R_CAP;
        Tout[0] = T0;
        Tout[1] = T1;
        Tout[2] = T2;
        return R_OK;
    }
    int rk = only < 0 ? 0 : only;
    const bool kept = !walked && T0 == n0 && nvis > 0 && rk == 0;
    bool reuse0 = kept && dir > 0.0 && T1 == vis[nvis - 1];
    bool chain = only < 0;  // no open fan so far: the shared-triangle shortcuts hold
    bool cwise = false;     // rotating clockwise through the rest of an open fan
    int x0 = -1;            // first apex of ring 0 (across edge T0-T2)
    int nrot = 0;           // apexes found by rotation in the current ring
    // Positions in S of T's vertices (tpk, packed) and of `cur` (always in
    // it): entries never move, so adding a bit to a vertex or apex whose
    // position is known needs no search.  The lists are those of S.add.
    int tpk = 0, cpos = -1;
    {
        const int f1 = rk == 2 ? 0 : rk + 1, f2 = rk == 0 ? 2 : rk - 1;
        if (!add_vertex(S, tpk, f1, tsel(f1), 1 << rk) || !add_vertex(S, tpk, f2, tsel(f2), 1 << rk)) return R_CAP;
        cur = tsel(f2);
        pcur = psel(f2);
        cpos = vertex_pos(tpk, f2);
    }
    if (kept && dir < 0.0 && nvis >= 2 && T2 == vis[nvis - 1]) {
        for (int s = nvis - 2; s >= 0; --s) {
            const int p = S.add(vis[s], 1);
            if (p < 0) return R_CAP;
            if (s == 0) cpos = p;  // vis[0] is a0
        }
        x0 = vis[nvis - 2];
        nrot = nvis - 1;
        cur = a0;
        pcur = pa0;
    }
    // one exit: the loop ends with res >= 0 (a single exit keeps the
    // compiler from copying the live values at every early return)
    int res = -1;
    for (int it = 0; it < 8 * KMAX && res < 0; ++it) {
        g.progress(it);
        const int f = rk == 2 ? 0 : rk + 1;
        const int first = tsel(f);
        const double2 pf = psel(f);
        const double2 pvk = psel(rk);
        bool closed = false;
        int pred = cur;  // apex preceding `first` when the ring closes
        int ppos = cpos;
        double2 ppred = pcur;
        int nt = -1;
        double2 pk = pcur;
        if (rk == 2 && chain && x0 >= 0 && cur == x0) {
            closed = true;  // ring 2 reached x0: the next apex is T[0]
        } else {
            const double sgn = cwise ? -1.0 : 1.0;
            const Key k = g.wrap(tsel(rk), pvk, cur, pcur, sgn);
            if (k.t == -2) {
                res = R_MORE;
                break;
            }
            nt = k.t;
            pk = make_double2(k.bx, k.by);
            if (cwise) {
                closed = nt < 0;
            } else if (nt < 0) {
                if (!g.global()) {
                    res = R_MORE;
                    break;
                }
                // open fan (hull vertex): the rest lies clockwise from `first`
                cwise = true;
                chain = false;
                reuse0 = false;
                cur = first;
                pcur = pf;
                cpos = vertex_pos(tpk, f);
                continue;
            } else {
                circumcircle<G::kFastCircle>(k, pvk, pcur, 1.0, cx, cy, rr);
                if (!g.certify(cx, cy, rr)) {
                    res = R_MORE;
                    break;
                }
                if (rk == 0 && reuse0) {
                    // co-circular ties can step past the stop: the turn is then complete
                    closed = nt == a0 || (orient(pvk, pcur, pa0) > 0.0 && orient(pvk, pa0, pk) > 0.0);
                    if (closed) {
                        for (int s = 0; s < nvis; ++s) {
                            const int p = S.add(vis[s], 1);
                            if (p < 0) {
                                res = R_CAP;
                                break;
                            }
                            if (s == nvis - 2) ppos = p;
                        }
                        if (res >= 0) break;
                        if (nvis >= 2) {
                            pred = vis[nvis - 2];
                            ppred = g.P(pred);
                        }
                    }
                } else {
                    closed = nt == first || (orient(pvk, pcur, pf) > 0.0 && orient(pvk, pf, pk) > 0.0);
                }
                if (!closed && rk == 0 && nrot == 0) x0 = nt;
            }
        }
        if (closed) {
            if (++rk == 3 || only >= 0) {
                res = R_OK;
                break;
            }
            cwise = false;
            const int f1 = rk == 2 ? 0 : rk + 1, f2 = rk == 0 ? 2 : rk - 1;
            if (!add_vertex(S, tpk, f1, tsel(f1), 1 << rk) || !add_vertex(S, tpk, f2, tsel(f2), 1 << rk)) {
                res = R_CAP;
                break;
            }
            if (chain && pred != tsel(f2)) {
                // the first apex of this ring is the one that preceded
                // `first` in the ring just closed (already in the list)
                S.set_bit(ppos, 1 << rk);
                cur = pred;
                pcur = ppred;
                cpos = ppos;
            } else {
                cur = tsel(f2);
                pcur = psel(f2);
                cpos = vertex_pos(tpk, f2);
            }
            nrot = 0;
        } else {
            const int p = S.add(nt, 1 << rk);
            if (p < 0) {
                res = R_CAP;
                break;
            }
            cur = nt;
            pcur = pk;
            cpos = p;
            ++nrot;
        }
    }
    if (res == R_OK) {
        Tout[0] = T0;
        Tout[1] = T1;
        Tout[2] = T2;
    }
    return res < 0 ? R_FAIL : res;
}

// ---------------------------------------------------------------- algebra
// (moment sums, Cholesky and the rank-revealing solver: algebra.h)

// Pseudo-inverse solve by cyclic Jacobi of the Gram matrix, for the mesh-side
// edge table (one thread per mesh edge; the systems of edges at the mesh
// boundary lose rank exactly, the others are well conditioned).  Eigenvalues
// below 1e-12 * lambda_max are dropped.
__device__ void pinv6_solve(const Moments& mo, const double b[6], double y[6]) {
    double Gl[6][6], A[6][6], V[6][6];
    mo.gram(Gl);
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

// Sum over the four lanes of a quad; every lane gets the same bits
// ((a+b)+(c+d) in all lanes, as FP addition is commutative).
__device__ __forceinline__ double quad_sum(double v) {
    v += lane_xor<QL>(v, 1);
    v += lane_xor<QL>(v, 2);
    return v;
}

// ------------------------------------------------------------ kernel args
struct KArgs {
    const double2* pos_s;
    const int32_t* perm;
    const int32_t* start;
    const SetDesc* sets;  // [S]
    int S;
    int levels;           // slow path: region doublings before the global scan
    int64_t n_nodes;      // all sets
    int64_t n_slots;      // ELL row slots of all sets (TILE_N per node tile)
    BuildOut out;
    int32_t* slow;        // slow-path list of row slots (capacity n_nodes)
    int32_t* rd;          // rank-deficient list of row slots (capacity n_nodes)
    int32_t* tdiag;       // [n_slots / TILE_N][5] per-tile counts of k_weights
    unsigned long long* diag;
    int linear;           // interior rows: barycentric coordinates in T only
    int per;              // periodic box: nearest images, no boundary ring
    double svd_kappa;     // a system whose estimate trace(G) trace(G^-1)
                          // exceeds this goes to the rank-revealing solver
};

// The set of a node tile / of a row slot.
__device__ __forceinline__ SetDesc tile_set(const KArgs& a, int64_t tile) {
    const int si = set_search(a.S, tile, [&](int s) { return a.sets[s].t0; });
    return a.sets[si];
}
__device__ __forceinline__ SetDesc slot_set(const KArgs& a, int64_t slot) { return tile_set(a, slot / TILE_N); }

__device__ __forceinline__ uint32_t pending_type(uint32_t t) { return t == NT_OUTSIDE ? NT_PEND_OUT : NT_PEND_RING; }

// Weights of one row by the rank-revealing solver, one wave per row, support
// entry k in lane k (KMAX <= WAVE).  Every system of the row is solved by
// one-sided Jacobi in the frame in which the conditions are stated:
//  * interior: for each edge e = (nu, sigma) of T, the rows of eqs. (A0),
//    (A1), (A2_2) relative to the edge ends, a = (r - r_nu) / s and
//    c = (r - r_sigma) / s with s = |r_nu - r_sigma|:
//    (1, a_x, a_y, a_x c_x, (a_x c_y + a_y c_x) / 2, a_y c_y) A = (0, 0, 0,
//    -d_x^2 / 2, -d_x d_y / 2, -d_y^2 / 2), d = (r_nu - r_sigma) / s;
//  * closure: the monomials of (r - q) / h against p(0).
// For a full-rank system the answer does not depend on the frame; below
// rank 6 the least-squares answer does, and this is the frame of the
// conditions as written.  Singular values below eps max(6, K) s_max are
// dropped.  Writes the finished row (user ids, weights, ring bits, meta);
// returns the number of systems solved, with the number of them below rank
// 6 in `nrd` and the largest cond2(G) of the full-rank ones in `kmax`.
template <bool PER>
__device__ int wave_row_svd(const KArgs& a, const SetDesc& sd, int64_t slot, double2 q, int lane, int& nrd,
                            double& kmax) {
    const int64_t nn = a.n_slots;
    const uint32_t meta = a.out.meta[slot];
    const uint32_t type = meta_type(meta);
    const int n = static_cast<int>(meta_cnt(meta));
    const bool in = lane < n;
    uint32_t e = 0;
    double2 p = make_double2(0.0, 0.0);
    int32_t uid = 0;
    // entries KMAX.. of a long row live in its overflow row
    const int32_t orow = n > KMAX ? a.out.orow[slot] : 0;
    const int64_t at = lane < KMAX ? lane * nn + slot : ovf_at(a.out.n_ovf, orow, lane);
    int32_t* const pidx = lane < KMAX ? a.out.idx : a.out.oidx;
    uint8_t* const pmem = lane < KMAX ? a.out.mem : a.out.omem;
    if (in) {
        e = static_cast<uint32_t>(pidx[at]) | (static_cast<uint32_t>(pmem[at]) << 28);
        const double2 r = a.pos_s[e & IDX_MASK];
        p = PER ? image_near(sd.m, r, q) : r;
        uid = a.perm[e & IDX_MASK];
    }
    uint32_t flags = meta_flags(meta) | MF_SVD;
    int nsys = 0;
    nrd = 0;
    kmax = 0.0;
    double w = 0.0;
    WaveSVD sv;
    if (type == NT_PENDING) {
        const int lt[3] = {static_cast<int>(meta_t(meta, 0)), static_cast<int>(meta_t(meta, 1)),
                           static_cast<int>(meta_t(meta, 2))};
        double2 P[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) P[k] = make_double2(lane_value(p.x, lt[k]), lane_value(p.y, lt[k]));
        // barycentric coordinates of q in T (linear FE, eqs. C0, C1)
        const double D = orient(P[0], P[1], P[2]);
        const double phi[3] = {orient(q, P[1], P[2]) / D, orient(P[0], q, P[2]) / D, orient(P[0], P[1], q) / D};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (lane == lt[k]) w += phi[k];
        if (!a.linear) {
#pragma unroll
            for (int ed = 0; ed < 3; ++ed) {
                const int pa = ed, pb = ed == 2 ? 0 : ed + 1;
                const double2 rn = P[pa], rs = P[pb];
                const double dxv = rn.x - rs.x, dyv = rn.y - rs.y;
                const double is = 1.0 / sqrt(dxv * dxv + dyv * dyv);
                const bool mem = in && (((e >> 28) >> pa) & 1u || ((e >> 28) >> pb) & 1u);
                const int keff = __popcll(__ballot(mem));
                const double ax = (p.x - rn.x) * is, ay = (p.y - rn.y) * is;
                const double cx = (p.x - rs.x) * is, cy = (p.y - rs.y) * is;
                sv.B[0] = mem ? 1.0 : 0.0;
                sv.B[1] = mem ? ax : 0.0;
                sv.B[2] = mem ? ay : 0.0;
                sv.B[3] = mem ? ax * cx : 0.0;
                sv.B[4] = mem ? 0.5 * (ax * cy + ay * cx) : 0.0;
                sv.B[5] = mem ? ay * cy : 0.0;
                wave_svd(sv, lane, keff);
                const double dx = dxv * is, dy = dyv * is;
                const double b[6] = {0.0, 0.0, 0.0, -0.5 * dx * dx, -0.5 * dx * dy, -0.5 * dy * dy};
                const double A = wave_svd_solve(sv, b, lane);
                if (mem) w += 2.0 * phi[pa] * phi[pb] * A;
                if (sv.rank < 6) {
                    flags |= MF_RANKDEF | (MF_RD0 << ed);
                    ++nrd;
                } else {
                    kmax = fmax(kmax, wave_svd_gram_cond(sv));
                }
                ++nsys;
            }
        }
    } else {
        // closure: minimum-norm weights of the quadratic moment conditions
        const double ih = 1.0 / sd.h;
        monos((p.x - q.x) * ih, (p.y - q.y) * ih, sv.B);
        if (!in) {
#pragma unroll
            for (int t = 0; t < 6; ++t) sv.B[t] = 0.0;
        }
        wave_svd(sv, lane, n);
        const double b[6] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        w = wave_svd_solve(sv, b, lane);
        if (sv.rank < 6) {
            flags |= MF_RANKDEF | MF_RD0;
            nrd = 1;
        } else {
            kmax = wave_svd_gram_cond(sv);
        }
        nsys = 1;
    }
    if (in) {
        double* const pw64 = lane < KMAX ? a.out.w64 : a.out.ow64;
        float* const pw32 = lane < KMAX ? a.out.w32 : a.out.ow32;
        pidx[at] = uid;
        pw64[at] = w;
        if (pw32) pw32[at] = static_cast<float>(w);
        pmem[at] = type == NT_PENDING ? static_cast<uint8_t>(e >> 28) : 0;
    }
    if (lane == 0) {
        const uint32_t ft = type == NT_PENDING ? NT_INTERIOR : (type == NT_PEND_OUT ? NT_OUTSIDE : NT_RING);
        a.out.meta[slot] = type == NT_PENDING ? meta_pack(ft, n, meta_t(meta, 0), meta_t(meta, 1), meta_t(meta, 2), flags)
                                              : meta_pack(ft, n, 0, 0, 0, flags);
    }
    return nsys;
}

// ------------------------------------------------------------ fast kernel
// One quad per node.  Interior nodes: certified Delaunay work in registers;
// the support goes to the ELL row as a PENDING row (sorted indices and ring
// bits) for k_weights.  Boundary-ring nodes: the KNN nearest particles,
// picked one per round (smallest squared distance, ties by user id), as a
// pending closure row.  Anything not certified goes to the slow list.
constexpr int TCAP = 1664;  // particles of a tile's bin region staged in LDS
constexpr int TDIM = 48;    // bin rows / columns of that region (at most)
constexpr int VPITCH = 16;  // wedge-search visit list per quad (longer: the exact path)

// Candidates in LDS fit 128 registers and 40 KB of LDS per block, so four
// waves per SIMD (four blocks per CU): the waves are bound by the latency of
// the dependent FP64 chains of the gift-wrapping steps, which more resident
// waves hide, and a 257 x 257 node mesh's 1024 full tiles run in one round.
template <int NS>
__global__ void __launch_bounds__(QWG) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_build_fast(KArgs a) {
    // highest issue priority until the rings (lowered as they progress)
    __builtin_amdgcn_s_setprio(3);
    // the tile's bin region (its nodes' search windows): bin starts, row
    // bases and the particles, copied once with coalesced row reads.  The
    // bin starts are needed only until every quad has gathered; the per-quad
    // support rows (padded by one word, so that the 16 quads of a wave hit
    // distinct LDS banks) take their place afterwards.
    constexpr int TSU = QPB * (KPITCH + VPITCH);
    constexpr int TSH = TDIM * (TDIM + 1) > TSU ? TDIM * (TDIM + 1) : TSU;
    __shared__ double2 tpos[TCAP];
    __shared__ int32_t tsh[TSH];
    __shared__ int32_t trb[TDIM + 1];
    __shared__ int32_t trs[TDIM];  // sorted index of each staged row's first particle
    int32_t* const tst = tsh;
    int32_t* const su = tsh;
    int32_t* const svis = tsh + QPB * KPITCH;
    const int lane = threadIdx.x & (QL - 1);
    const int qi = threadIdx.x / QL;
    const SetDesc sd = tile_set(a, blockIdx.x);
    int tx, ty;
    tile_xy(sd, static_cast<int>(blockIdx.x - sd.t0), tx, ty);
    // A tile holding the left or right boundary column takes its nodes
    // column by column: that column's ring nodes (the closure path) then
    // share one wave instead of adding their path to every wave of the tile.
    // The rows go to the same slots either way.
    const bool bycol = tx == 0 || tx * 8 + 7 >= sd.m.nx;
    const int lx = bycol ? (qi >> 3) : (qi & 7), ly = bycol ? (qi & 7) : (qi >> 3);
    const int i = tx * 8 + lx, j = ty * 8 + ly;
    const bool valid = i <= sd.m.nx && j <= sd.m.ny;
    const int slot = static_cast<int>(blockIdx.x) * TILE_N + ly * 8 + lx;  // < 2^31, checked on the host
    const int64_t nn = a.n_slots;
    const bool per = a.per != 0;
    const bool ring = !per && (i == 0 || j == 0 || i == sd.m.nx || j == sd.m.ny);
    const int32_t* start = a.start + sd.b0;
    bool done = false;
    // ---- stage the region (block-uniform decision): it covers the window
    // of every node of the tile, interior, edge or corner
    const int hcor = static_cast<int>(ceil(sd.Rc * 1.4142135623730951 / sd.g.bw));
    const bool xedge = tx == 0 || tx * 8 + 7 >= sd.m.nx, yedge = ty == 0 || ty * 8 + 7 >= sd.m.ny;
    const int hmax = per ? sd.hwf
                         : (xedge && yedge) ? max(max(sd.hwf, sd.hwc), hcor)
                                            : (xedge || yedge) ? max(sd.hwf, sd.hwc) : sd.hwf;
    const int rbx0 = max(tx * 8 * sd.g.kb - hmax, 0);
    const int rbx1 = min(min(tx * 8 + 7, sd.m.nx) * sd.g.kb + hmax, sd.g.nbx);
    const int rby0 = max(ty * 8 * sd.g.kb - hmax, 0);
    const int rby1 = min(min(ty * 8 + 7, sd.m.ny) * sd.g.kb + hmax, sd.g.nby);
    const int ncol = rbx1 - rbx0, nrow = rby1 - rby0;
    bool staged = ncol <= TDIM && nrow <= TDIM;
    if (staged) {
        {
            // a thread's bin starts all in flight before the first is stored
            constexpr int SPT = (TDIM * (TDIM + 1) + QWG - 1) / QWG;
            const int nst = nrow * (ncol + 1);
            int sv[SPT], sat[SPT];
#pragma unroll
            for (int u = 0; u < SPT; ++u) {
                const int e = static_cast<int>(threadIdx.x) + u * QWG;
                const int r = e / (ncol + 1), c = e - r * (ncol + 1);
                // (entries past the table load bin 0 and are not stored)
                sat[u] = e < nst ? r * (TDIM + 1) + c : -1;
                sv[u] = start[e < nst ? (rby0 + r) * sd.g.nbx + rbx0 + c : 0];
            }
#pragma unroll
            for (int u = 0; u < SPT; ++u)
                if (sat[u] >= 0) tst[sat[u]] = sv[u];
        }
        __syncthreads();
        if (threadIdx.x < WAVE) {
            // row bases: an exclusive prefix sum of the row lengths over the
            // first wave (nrow <= TDIM < 64 rows)
            const int r = threadIdx.x;
            const int len = r < nrow ? tst[r * (TDIM + 1) + ncol] - tst[r * (TDIM + 1)] : 0;
            int inc = len;
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                const int o = __shfl_up(inc, d);
                if (r >= d) inc += o;
            }
            if (r <= nrow) trb[r] = inc - len;
            if (r < nrow) trs[r] = tst[r * (TDIM + 1)];
        }
        __syncthreads();
        const int total = trb[nrow];
        staged = total <= TCAP;
        if (staged) {
            // every source index first, then all loads in flight together
            // (entries past the total load particle 0 and are not stored)
            constexpr int EPT = (TCAP + QWG - 1) / QWG;
            int src[EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = static_cast<int>(threadIdx.x) + u * QWG;
                int lo = 0, hi = nrow - 1;  // the row holding staged entry e
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (trb[mid] <= e) lo = mid;
                    else hi = mid - 1;
                }
                src[u] = e < total ? tst[lo * (TDIM + 1)] + (e - trb[lo]) : 0;
            }
            double px[EPT], py[EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const double2 v = a.pos_s[src[u]];
                px[u] = v.x;
                py[u] = v.y;
            }
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = static_cast<int>(threadIdx.x) + u * QWG;
                if (e < total) tpos[e] = make_double2(px[u], py[u]);
            }
        }
        __syncthreads();
    }
    QuadSource<NS> g;
    g.perm = a.perm;
    g.lpos = tpos;
    g.lrb = trb;
    g.lrs = trs;
    g.nrow = nrow;
#pragma unroll
    for (int k = 0; k < (NS + 1) / 2; ++k) g.ci_[k] = 0u;
    g.n = 0;
    g.lane = lane;
    // a region too large to stage leaves its nodes to the exact path
    int ovf = staged ? 0 : 1;
    if (valid && staged) {
        g.q = node_at(sd.m, i, j, per);
        // a corner node sees a quarter disk, an edge node a half disk: the
        // corner radius is sqrt(2) larger for the same expected count
        const bool corner = (i == 0 || i == sd.m.nx) && (j == 0 || j == sd.m.ny);
        g.Rf = ring ? (corner ? sd.Rc * 1.4142135623730951 : sd.Rc) : sd.Rf;
        // gather the particles within the radius.  The quad walks each row
        // segment of the window four particles at a time; the k-th particle
        // accepted (in the order of the walk) goes to lane k % 4, so that no
        // lane holds more than ceil(n / 4) of the node's n candidates.
        const double R2 = g.Rf * g.Rf;
        const int hw = ring ? (corner ? static_cast<int>(ceil(g.Rf / sd.g.bw)) : sd.hwc) : sd.hwf;
        const int cbx = i * sd.g.kb, cby = j * sd.g.kb;
        const int bx0 = max(cbx - hw, 0), bx1 = min(cbx + hw, sd.g.nbx);
        const int by0 = max(cby - hw, 0), by1 = min(cby + hw, sd.g.nby);
        // in a periodic box a node runs here only when its window stays a bin
        // inside the box sides (its particles are then their own nearest
        // images and no image lies in the window); the others take the exact
        // path, whose regions wrap
        if (per && (cbx - hw < 1 || cbx + hw > sd.g.nbx - 1 || cby - hw < 1 || cby + hw > sd.g.nby - 1)) ovf = 1;
        int acc = 0;  // particles accepted so far (the same in the four lanes)
        auto insert = [&](int t) {
            if (g.n >= NS) {
                ovf = 1;
                return;
            }
            // every word rewritten through a select: a store at a run-time
            // index would put the array in scratch memory
            const uint32_t bits = static_cast<uint32_t>(t) << ((g.n & 1) << 4);
            const int word = g.n >> 1;
#pragma unroll
            for (int k = 0; k < (NS + 1) / 2; ++k) g.ci_[k] = k == word ? (g.ci_[k] | bits) : g.ci_[k];
            ++g.n;
        };
        // staged particles s .. e - 1 of one row segment
        auto segment = [&](int s, int e) {
            for (int t0 = s; t0 < e; t0 += QL) {
                const int t = t0 + lane;
                bool in = false;
                if (t < e) {
                    const double2 p = tpos[t];
                    const double dx = p.x - g.q.x, dy = p.y - g.q.y;
                    in = dx * dx + dy * dy <= R2;
                }
                int m = in ? 1 << lane : 0;
                m |= lane_xor<QL>(m, 1);
                m |= lane_xor<QL>(m, 2);
                const int c = __popc(m);
                const int k = (lane - acc) & (QL - 1);
                if (k < c) {
                    int mm = m;  // the k-th set bit of m
                    for (int r = 0; r < k; ++r) mm &= mm - 1;
                    insert(t0 + __ffs(mm) - 1);
                }
                acc += c;
            }
        };
        for (int by = by0; by < (ovf ? by0 : by1); ++by) {
            const int* rs = tst + (by - rby0) * (TDIM + 1);
            const int base = trb[by - rby0] - rs[0];
            segment(base + rs[bx0 - rbx0], base + rs[bx1 - rbx0]);
        }
    }
    __syncthreads();  // every quad has gathered: the support rows replace the bin starts
    // (an overflowed lane holds NS candidates too: it only keeps the slot)
    g.use_last = __ballot(valid && !ring && g.n >= NS) != 0;
    if (valid) {
        ovf |= lane_xor<QL>(ovf, 1);
        ovf |= lane_xor<QL>(ovf, 2);
        if (!ovf && !ring) {
            int T[3] = {0, 0, 0};
            Support<QL> S;
            S.u = su + qi * KPITCH;
            S.n = 0;
            S.lane = lane;
            const int st = delaunay_node(g, g.q, T, S, svis + qi * VPITCH, a.linear ? -2 : -1, VPITCH);
            if (st == R_OK) {
                const int lt0 = S.find(T[0]), lt1 = S.find(T[1]), lt2 = S.find(T[2]);
                if (lt0 >= 0 && lt1 >= 0 && lt2 >= 0) {
                    for (int k = lane; k < S.n; k += QL) {
                        const uint32_t e = static_cast<uint32_t>(S.u[k]);
                        a.out.idx[k * nn + slot] = g.sorted(static_cast<int>(e & IDX_MASK));
                        a.out.mem[k * nn + slot] = static_cast<uint8_t>(e >> 28);
                    }
                    if (lane == 0) a.out.meta[slot] = meta_pack(NT_PENDING, S.n, lt0, lt1, lt2, 0u);
                    done = true;
                }
            }
        } else if (!ovf) {
            // (after the rings of the wave's interior nodes, if any: the
            // waves that hold ring nodes are a tile's longest, so this part
            // takes the highest priority again)
            __builtin_amdgcn_s_setprio(3);
            // the KNN nearest candidates in the order of (d^2, user id).
            // Every slot's distance is computed once (slots past n: +inf);
            // the picks wait in the quad's support row (free on this path)
            // until the selection is over.
            double d2s[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const double2 b = tpos[g.cand(s)];  // slots past n hold index 0
                const double dx = b.x - g.q.x, dy = b.y - g.q.y;
                d2s[s] = s < g.n ? dx * dx + dy * dy : INFINITY;
            }
            int32_t* const picks = su + qi * KPITCH;
            // A candidate's place in that order is the number of the quad's
            // candidates strictly nearer, when no two distances are equal:
            // the KNN places are then written at once, with no chain of
            // rounds.  Equal distances give equal places; the quad sees that
            // (fewer distinct places than candidates placed) and takes the
            // rounds below, which break ties by user id.
            int place[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) place[s] = 0;
#pragma unroll
            for (int m = 0; m < QL; ++m)
#pragma unroll
                for (int so = 0; so < NS; ++so) {
                    const double od = m == 0 ? d2s[so] : lane_xor<QL>(d2s[so], m);
#pragma unroll
                    for (int s = 0; s < NS; ++s) place[s] += od < d2s[s] ? 1 : 0;
                }
            int hit = 0, placed = 0;
            double pd = -1.0;
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (s < g.n && place[s] < KNN) {
                    picks[place[s]] = g.cand(s);
                    hit |= 1 << place[s];
                    ++placed;
                    pd = fmax(pd, d2s[s]);
                }
#pragma unroll
            for (int m = 1; m < QL; m <<= 1) {
                hit |= lane_xor<QL>(hit, m);
                placed += lane_xor<QL>(placed, m);
                pd = fmax(pd, lane_xor<QL>(pd, m));
            }
            int found = placed;
            int pt = -1;
            if (__popc(static_cast<unsigned>(hit)) != placed) {
                found = 0;
                pd = -1.0;
            }
            for (int r = found > 0 || placed == 0 ? KNN : 0; r < KNN; ++r) {
                double bd = INFINITY;
                int bt = -1;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (s >= g.n) continue;
                    const int t = g.cand(s);
                    const double d2 = d2s[s];
                    const bool after = d2 > pd || (d2 == pd && t != pt && g.uid(t) > g.uid(pt));
                    const bool better = d2 < bd || (d2 == bd && bt >= 0 && g.uid(t) < g.uid(bt));
                    if (after && better) {
                        bd = d2;
                        bt = t;
                    }
                }
#pragma unroll
                for (int m = 1; m < QL; m <<= 1) {
                    const double od = lane_xor<QL>(bd, m);
                    const int ot = lane_xor<QL>(bt, m);
                    if (ot >= 0 && ot != bt && (bt < 0 || od < bd || (od == bd && g.uid(ot) < g.uid(bt)))) {
                        bd = od;
                        bt = ot;
                    }
                }
                if (bt < 0) break;
                if (lane == 0) picks[r] = bt;
                pd = bd;
                pt = bt;
                ++found;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int k = lane; k < found; k += QL) {
                a.out.idx[k * nn + slot] = g.sorted(picks[k]);
                a.out.mem[k * nn + slot] = 0;
            }
            // certified when the K-th distance is inside the gathered disk
            if (found == KNN && sqrt(pd) <= g.Rf * (1.0 - 1e-12)) {
                if (lane == 0) a.out.meta[slot] = meta_pack(NT_PEND_RING, KNN, 0, 0, 0, 0u);
                done = true;
            }
        }
    }
    if (!valid && lane == 0) a.out.meta[slot] = meta_pack(NT_FAILED, 0, 0, 0, 0, 0u);  // beyond the mesh
    if (valid && !done && lane == 0) {
        // an empty row until the slow path (or, for a periodic box's seam
        // node, k_seam_copy) writes it, so that no node is ever left with the
        // metadata of an earlier build (or of fresh memory)
        a.out.meta[slot] = meta_pack(NT_FAILED, 0, 0, 0, 0, 0u);
        if (!(per && (i == sd.m.nx || j == sd.m.ny))) {
            const int lpos = static_cast<int>(atomicAdd(&a.diag[D_SLOWCNT], 1ull));
            a.slow[lpos] = static_cast<int32_t>(slot);
        }
    }
}

// ------------------------------------------------------------ slow kernel
// Weights of every pending row (interior or closure, from either path), one
// quad per node, nodes in the same 8 x 8 tiles as the fast kernel.  Lanes
// 0..2 of a quad each own one edge system of the node's triangle (moments,
// Cholesky, one refinement step), lane 3 the barycentric part; the weights
// are quad sums per support entry.  The support's positions are staged in
// LDS.  A node with a rank-deficient system is left pending and listed for
// k_weights_rd (pseudo-inverse), which keeps this kernel's registers low.
constexpr int SK = 16;       // support entries staged in LDS per node
constexpr int SKP = SK + 1;  // row pitch: conflict-free LDS banks across quads

// The rows a weights pass owns: the fast path's (written before the pass
// starts) or the slow path's (flagged MF_ESCALATED, finished on the side
// stream while the fast rows are being weighted).
// Diagnostic counts of one wave's rows: interior, closure and outside-hull
// rows, and the largest support.
// Per-tile record of the weights pass: the four counts, then the largest
// condition estimate (FP32 bits).
constexpr int TD = BUILD_TD, TD_KMAX = 4;
static_assert(TD == 5, "four counts and the condition estimate");
struct WaveCounts {
    int c[4];
    float kmax;  // largest condition estimate of a system solved by Cholesky
};
enum { WC_INTERIOR, WC_CLOSURE, WC_OUTSIDE, WC_SUPMAX };

// QS quads may share one row (quad `sub` of them): each computes the whole
// row's systems, identically, and they split the final pass over the support
// entries (quad sub takes entries sub, sub + QS, ...), whose weights do not
// depend on one another, so the row is the same bit for bit for any QS.
// What the weights pass does with a finished row: store its weights in the
// handle's rows (StoreRows), or add them into the node's weighted sum of
// eq. (p2m) at once and store that (ProjRows: the fused build, which keeps
// no weights of these rows).
struct StoreRows {
    static constexpr bool proj = false;
};
template <typename TV, typename TW, typename TO, int CC>
struct ProjRows {
    static constexpr bool proj = true;
    using Sum = RowSum<TV, TW, TO, CC>;
    using W = TW;
    const TV* vals;
    TO* out;
    int C;
};

template <bool PER, int QS = 1, class R = StoreRows>
__device__ __forceinline__ WaveCounts weights_node(const KArgs& a, const SetDesc& sd, int i, int j, bool valid,
                                                   int64_t slot, int lane, int qi, double2* sp, uint32_t* se,
                                                   int32_t* su, bool escalated_rows, int sub = 0,
                                                   const R& rp = R{}, int* svd_here = nullptr) {
    static_assert(!R::proj || QS == 1, "a projected row is summed by one quad");
    const int64_t nn = a.n_slots;
    const uint32_t meta = valid ? a.out.meta[slot] : 0u;
    const bool mine = valid && (((meta_flags(meta) & MF_ESCALATED) != 0) == escalated_rows);
    const uint32_t type = mine ? meta_type(meta) : NT_FAILED;
    const int n = static_cast<int>(meta_cnt(meta));
    const bool pend = type == NT_PENDING;
    const bool clos = type == NT_PEND_RING || type == NT_PEND_OUT;
    const double2 q = node_at(sd.m, i, j, PER);
    auto img = [&](double2 p) { return PER ? image_near(sd.m, p, q) : p; };
    // stage the support: entry (sorted index | ring bits << 28), position and
    // user id.  The loads are unconditional, so that all of them are issued
    // before any is waited for: entries past the row (k < SK <= KMAX stays
    // inside the row storage) are replaced by particle 0 and not stored.
    {
        constexpr int SS = SK / QL;
        uint32_t e[SS];
        const int ns = (pend || clos) ? min(n, SK) : 0;
#pragma unroll
        for (int s = 0; s < SS; ++s) {
            const int k = s * QL + lane;
            const uint32_t v = static_cast<uint32_t>(a.out.idx[k * nn + slot]) |
                               (static_cast<uint32_t>(a.out.mem[k * nn + slot]) << 28);
            e[s] = k < ns ? v : 0u;
        }
        double2 pp[SS];
        int32_t uu[SS];
#pragma unroll
        for (int s = 0; s < SS; ++s) {
            pp[s] = img(a.pos_s[e[s] & IDX_MASK]);
            uu[s] = a.perm[e[s] & IDX_MASK];
        }
#pragma unroll
        for (int s = 0; s < SS; ++s) {
            const int k = s * QL + lane;
            if (k < ns) {
                se[qi * SKP + k] = e[s];
                sp[qi * SKP + k] = pp[s];
                su[qi * SKP + k] = uu[s];
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // weights pass: issue priority lowered as a wave advances (staged, then
    // solved), so that a CU's later blocks (its last, a boundary tile's
    // closure rows) are not held back by the older ones; the exact path
    // keeps the highest priority throughout
    if (!escalated_rows) __builtin_amdgcn_s_setprio(2);
    // f(k, entry, position, user id) over the support: staged slots from LDS,
    // the rest (rare) from global memory, in two loops so that neither
    // needs a generic (flat) address
    auto each = [&](auto&& f) {
        const int ns = min(n, SK);
#pragma unroll 4
        for (int k = 0; k < ns; ++k) f(k, se[qi * SKP + k], sp[qi * SKP + k], su[qi * SKP + k]);
        for (int k = SK; k < n; ++k) {
            const uint32_t e = static_cast<uint32_t>(a.out.idx[k * nn + slot]) |
                               (static_cast<uint32_t>(a.out.mem[k * nn + slot]) << 28);
            f(k, e, img(a.pos_s[e & IDX_MASK]), a.perm[e & IDX_MASK]);
        }
    };
    auto P = [&](int k) -> double2 {
        if (k < SK) return sp[qi * SKP + k];
        return img(a.pos_s[a.out.idx[k * nn + slot]]);
    };
    int ok = 1;
    double kap = 0.0;  // condition estimate of this lane's system
    double y[6] = {0, 0, 0, 0, 0, 0};
    // edge / closure frame: x~ = (p - c) * s
    double cx = 0.0, cy = 0.0, sc = 1.0, coef = 0.0;
    int mask = 0;
    double phi[3] = {0, 0, 0};
    int lt[3] = {0, 0, 0};
    if (pend) {
#pragma unroll
        for (int k = 0; k < 3; ++k) lt[k] = static_cast<int>(meta_t(meta, k));
        const double2 P0 = P(lt[0]), P1 = P(lt[1]), P2 = P(lt[2]);
        // barycentric coordinates of q in T (linear FE, eqs. C0, C1)
        const double D = orient(P0, P1, P2);
        phi[0] = orient(q, P1, P2) / D;
        phi[1] = orient(P0, q, P2) / D;
        phi[2] = orient(P0, P1, q) / D;
        if (lane < 3 && !a.linear) {
            const int pb = lane == 2 ? 0 : lane + 1;
            const double2 rn = lane == 0 ? P0 : (lane == 1 ? P1 : P2);
            const double2 rs = pb == 0 ? P0 : (pb == 1 ? P1 : P2);
            cx = 0.5 * (rn.x + rs.x);
            cy = 0.5 * (rn.y + rs.y);
            const double dxv = rn.x - rs.x, dyv = rn.y - rs.y;
            sc = 1.0 / sqrt(dxv * dxv + dyv * dyv);
            mask = (1 << lane) | (1 << pb);
            // selected by value: a run-time index would put phi in scratch
            const double pa_ = lane == 0 ? phi[0] : (lane == 1 ? phi[1] : phi[2]);
            const double pb_ = pb == 0 ? phi[0] : (pb == 1 ? phi[1] : phi[2]);
            coef = 2.0 * pa_ * pb_;
            const double dx = dxv * sc, dy = dyv * sc;
            // eq. A2_2 in the edge frame (eqs. A0, A1 give the zero rows)
            const double b[6] = {0.0, 0.0, 0.0, -0.5 * dx * dx, -0.5 * dx * dy, -0.5 * dy * dy};
            Moments mo;
            mo.zero();
            each([&](int, uint32_t e, double2 p, int32_t) {
                if ((e >> 28) & mask) mo.add((p.x - cx) * sc, (p.y - cy) * sc);
            });
            double L[6][6];
            mo.gram(L);
            const double tr = mo.trace();
            ok = chol6(L) ? 1 : 0;
            if (ok) {
                // ill-conditioned systems go to the rank-revealing solver
                kap = tr * chol6_inv_trace(L);
                if (!(kap <= a.svd_kappa)) ok = 0;
            }
            if (ok) {
                chol6_solve(L, b, y);
                double r[6] = {0, 0, 0, 0, 0, 0};
                each([&](int, uint32_t e, double2 p, int32_t) {
                    if (!((e >> 28) & mask)) return;
                    double pm[6];
                    monos((p.x - cx) * sc, (p.y - cy) * sc, pm);
                    const double A = dot6(pm, y);
#pragma unroll
                    for (int t = 0; t < 6; ++t) r[t] += A * pm[t];
                });
#pragma unroll
                for (int t = 0; t < 6; ++t) r[t] = b[t] - r[t];
                double d[6];
                chol6_solve(L, r, d);
#pragma unroll
                for (int t = 0; t < 6; ++t) y[t] += d[t];
            }
        }
    } else if (clos) {
        // minimum-norm quadratic moment conditions over the nearest
        // particles, centred at their centroid and scaled by their RMS radius.
        // The four lanes share every pass over the entries (lane l takes
        // entries l, l + 4, ...; quad sums), so all of them hold the solution.
        auto each4 = [&](auto&& f) {
            const int ns = min(n, SK);
            for (int k = lane; k < ns; k += QL) f(sp[qi * SKP + k]);
            for (int k = SK + lane; k < n; k += QL) f(P(k));
        };
        double sx = 0.0, sy = 0.0;
        each4([&](double2 p) {
            sx += p.x;
            sy += p.y;
        });
        cx = quad_sum(sx) / n;
        cy = quad_sum(sy) / n;
        double r2 = 0.0;
        each4([&](double2 p) { r2 += (p.x - cx) * (p.x - cx) + (p.y - cy) * (p.y - cy); });
        r2 = quad_sum(r2);
        sc = r2 > 0.0 ? 1.0 / sqrt(r2 / n) : 1.0;
        Moments mo;
        mo.zero();
        each4([&](double2 p) { mo.add((p.x - cx) * sc, (p.y - cy) * sc); });
#pragma unroll
        for (int t = 0; t < 15; ++t) mo.m[t] = quad_sum(mo.m[t]);
        double b[6];
        monos((q.x - cx) * sc, (q.y - cy) * sc, b);
        double L[6][6];
        mo.gram(L);
        const double tr = mo.trace();
        ok = chol6(L) ? 1 : 0;
        if (ok) {
            kap = tr * chol6_inv_trace(L);
            if (!(kap <= a.svd_kappa)) ok = 0;
        }
        if (ok) {
            chol6_solve(L, b, y);
            double r[6] = {0, 0, 0, 0, 0, 0};
            each4([&](double2 p) {
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
        }
        coef = 1.0;
    }
    if (!escalated_rows) __builtin_amdgcn_s_setprio(1);
    ok = min(ok, lane_xor<QL>(ok, 1));
    ok = min(ok, lane_xor<QL>(ok, 2));
    if ((pend || clos) && !ok) {
        // ill-conditioned or rank-deficient: the row stays pending for the
        // rank-revealing solver (k_weights_rd), or, with svd_here, for the
        // caller to solve that way at once
        if (svd_here) {
            *svd_here = 1;
        } else if (lane == 0 && sub == 0) {
            const int lpos = static_cast<int>(atomicAdd(&a.diag[D_RDCNT], 1ull));
            a.rd[lpos] = static_cast<int32_t>(slot);
        }
    } else if (pend || clos) {
        // w_k = phi-part (lane 3) + sum over the edges (lanes 0..2) of
        // 2 phi_nu phi_sigma A_{e,k}; closure: lane k mod 4 alone
        auto each_sub = [&](auto&& f) {
            const int ns = min(n, SK);
            for (int k = sub; k < ns; k += QS) f(k, se[qi * SKP + k], sp[qi * SKP + k], su[qi * SKP + k]);
            for (int k = SK + sub; k < n; k += QS) {
                const uint32_t e = static_cast<uint32_t>(a.out.idx[k * nn + slot]) |
                                   (static_cast<uint32_t>(a.out.mem[k * nn + slot]) << 28);
                f(k, e, img(a.pos_s[e & IDX_MASK]), a.perm[e & IDX_MASK]);
            }
        };
        auto weight = [&](int k, uint32_t e, double2 p) {
            double c = 0.0;
            if (pend && lane == 3) {
                c = (k == lt[0] ? phi[0] : 0.0) + (k == lt[1] ? phi[1] : 0.0) + (k == lt[2] ? phi[2] : 0.0);
            } else if (clos ? lane == (k & (QL - 1)) : (lane < 3 && ((e >> 28) & mask))) {
                double pm[6];
                monos((p.x - cx) * sc, (p.y - cy) * sc, pm);
                c = coef * dot6(pm, y);
            }
            return quad_sum(c);
        };
        if constexpr (R::proj) {
            // lane k % 4 adds entry k, in ascending k: the order of the
            // stored-weights projection
            typename R::Sum rs;
            rs.init();
            each_sub([&](int k, uint32_t e, double2 p, int32_t u) {
                const double w = weight(k, e, p);
                if (lane == (k & (QL - 1))) rs.add(static_cast<typename R::W>(w), rp.vals, u, rp.C);
            });
            rs.store(rp.out, ij_node(sd, i, j), rp.C, lane);
        } else {
            each_sub([&](int k, uint32_t e, double2 p, int32_t u) {
                const double w = weight(k, e, p);
                if (lane == (k & (QL - 1))) {
                    a.out.idx[k * nn + slot] = u;
                    a.out.w64[k * nn + slot] = w;
                    if (a.out.w32) a.out.w32[k * nn + slot] = static_cast<float>(w);
                    a.out.mem[k * nn + slot] = clos ? 0 : static_cast<uint8_t>(e >> 28);
                }
            });
        }
        if (lane == 0 && sub == 0) {
            const uint32_t ft = pend ? NT_INTERIOR : (type == NT_PEND_OUT ? NT_OUTSIDE : NT_RING);
            a.out.meta[slot] = pend ? meta_pack(ft, n, lt[0], lt[1], lt[2], meta_flags(meta))
                                    : meta_pack(ft, n, 0, 0, 0, meta_flags(meta));
        }
    }
    // diagnostics: one count per row (lane 0 of quad 0), wave-uniform totals
    const bool q0 = lane == 0 && sub == 0;
    WaveCounts wc;
    wc.c[WC_INTERIOR] = __popcll(__ballot(q0 && pend));
    wc.c[WC_CLOSURE] = __popcll(__ballot(q0 && clos));
    wc.c[WC_OUTSIDE] = __popcll(__ballot(q0 && type == NT_PEND_OUT));
    int sup = (pend || clos) ? n : 0;
    for (int off = 32; off > 0; off >>= 1) sup = max(sup, __shfl_xor(sup, off));
    wc.c[WC_SUPMAX] = sup;
    float kf = ((pend || clos) && ok) ? static_cast<float>(kap) : 0.0f;
    for (int off = 32; off > 0; off >>= 1) kf = fmaxf(kf, __shfl_xor(kf, off));
    wc.kmax = kf;
    return wc;
}

// Adds one wave's counts to the diagnostics (the few slow-path rows).
__device__ __forceinline__ void count_wave(const KArgs& a, const WaveCounts& wc) {
    if (threadIdx.x % WAVE != 0) return;
    if (wc.c[WC_INTERIOR]) atomicAdd(&a.diag[D_INTERIOR], static_cast<unsigned long long>(wc.c[WC_INTERIOR]));
    if (wc.c[WC_CLOSURE]) atomicAdd(&a.diag[D_CLOSURE], static_cast<unsigned long long>(wc.c[WC_CLOSURE]));
    if (wc.c[WC_OUTSIDE]) atomicAdd(&a.diag[D_OUTSIDE], static_cast<unsigned long long>(wc.c[WC_OUTSIDE]));
    if (wc.c[WC_SUPMAX]) atomicMax(&a.diag[D_SUPMAX], static_cast<unsigned long long>(wc.c[WC_SUPMAX]));
    if (wc.kmax > 0.0f)
        atomicMax(&a.diag[D_GRAMCOND],
                  static_cast<unsigned long long>(__double_as_longlong(static_cast<double>(wc.kmax))));
}

// One wave per listed node: certified Delaunay search (exact predicates)
// over square bin regions that double in half-width up to every particle;
// interior nodes leave their support in the ELL row, closure nodes (ring, or
// outside the hull) their nearest particles; k_weights does the rest.
// LDS of the exact path's node loop: visit lists, staged regions and ring
// lists of its three waves, and (when it weighs its rows) the row staging.
struct SlowLds {
    int32_t* svis;   // [3 * KROW]
    double2* slp;    // [3 * STAGE]
    int32_t* slt;    // [3 * STAGE]
    int32_t* sring;  // [3 * KROW]
    int* sinfo;      // [3 * 3]
    double2* wsp;    // [(WAVE / QL) * SKP] (weighing only)
    uint32_t* wse;
    int32_t* wsu;
};

template <bool PER, bool WEIGH>
__device__ __forceinline__ void slow_nodes(const KArgs& a, int first, int stride, const SlowLds& L) {
    constexpr int WPB = SWG / WAVE;
    static_assert(WPB == 3, "one wave per ring");
    int32_t* const svis = L.svis;
    double2* const slp = L.slp;
    int32_t* const slt = L.slt;
    // These few waves are a serial latency chain beside the weights pass:
    // they take issue priority over its waves.
    __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x & (WAVE - 1);
    // the wave's index, read as a scalar: every value derived from it (the
    // node, its position, its search) is then visibly wave-uniform and its
    // branches stay scalar
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / WAVE));
    const int count = static_cast<int>(a.diag[D_SLOWCNT]);
    const int64_t nn = a.n_slots;
    for (int li = first; li < count; li += stride) {
        // the previous node's lists have been read
        __syncthreads();
        const int64_t slot = a.slow[li];
        const SetDesc sd = slot_set(a, slot);
        const int big = max(sd.g.nbx, sd.g.nby) + 1;
        int i, j;
        slot_ij(sd, slot, i, j);
        constexpr bool per = PER;
        const double2 q = node_at(sd.m, i, j, per);
        const bool ring = !per && (i == 0 || j == 0 || i == sd.m.nx || j == sd.m.ny);
        const int cbx = (per && i == sd.m.nx ? 0 : i) * sd.g.kb, cby = (per && j == sd.m.ny ? 0 : j) * sd.g.kb;
        // (the launch that shares its blocks with the weights pass keeps the
        // regions in LDS: its register budget is the weights pass's)
        WaveSource<PER, WEIGH> c;
        c.pos = a.pos_s;
        c.perm = a.perm;
        c.start = a.start + sd.b0;
        c.g = sd.g;
        c.m = sd.m;
        c.q = q;
        c.neardeg = 0;
        c.ring_mark = 0;
        c.lane = lane;
        // (a fourth wave of a block takes part in its barriers only)
        c.lp = slp + min(wv, WPB - 1) * STAGE;
        c.lt = slt + min(wv, WPB - 1) * STAGE;
        static_assert(KROW <= WAVE, "one support entry per lane");
        WaveSupport S;
        S.e = 0;
        S.n = 0;
        S.lane = lane;
        uint32_t type = ring ? NT_RING : NT_INTERIOR;
        uint32_t flags = MF_ESCALATED;
        int T[3] = {0, 0, 0};
        int st = R_FAIL;
        int ndeg = 0;  // near ties of the node, over its three waves
        if (!ring) {
            // wave k finds the triangle and then the ring of its vertex k
            for (int level = 0;; ++level) {
                const int hw = level < a.levels ? (sd.hw0 << level) : big;
                const Region reg = per ? make_region_periodic(sd.g, cbx, cby, hw) : make_region(sd.g, cbx, cby, hw);
                if (wv < WPB) {
                    c.set_region(reg);
                    S.n = 0;
                    const int sk = delaunay_node(c, q, T, S, svis + wv * KROW, a.linear ? -2 : wv, KROW);
                    if (lane < S.n) L.sring[wv * KROW + lane] = S.e;
                    if (lane == 0) {
                        L.sinfo[wv * 3] = sk;
                        L.sinfo[wv * 3 + 1] = S.n;
                        // the wedge and walk counted once, by the ring-0 wave
                        L.sinfo[wv * 3 + 2] = wv == 0 ? c.neardeg : c.neardeg - c.ring_mark;
                    }
                } else {
                    c.R = reg;
                }
                __syncthreads();
                // the chained routine returns the first failure in ring order
                st = R_OK;
                for (int w = 0; w < WPB; ++w)
                    if (st == R_OK) st = L.sinfo[w * 3];
                ndeg = L.sinfo[2] + L.sinfo[5] + L.sinfo[8];
                if (st != R_MORE) break;
                __syncthreads();  // every wave has read this level's results
                if (c.R.global) {
                    st = R_FAIL;
                    break;
                }
            }
        }
        // the rest of the node is the ring-0 wave's
        if (wv != 0) continue;
        if (st == R_OK) {
            // ring 0's list, then the new entries of rings 1 and 2 in their
            // order (ring bits of shared entries OR-ed): the chained order
            for (int w = 1; w < WPB && st == R_OK; ++w)
                for (int k = 0; k < L.sinfo[w * 3 + 1]; ++k) {
                    const uint32_t e = static_cast<uint32_t>(L.sring[w * KROW + k]);
                    if (S.add(static_cast<int>(e & IDX_MASK), static_cast<int>(e >> 28)) < 0) {
                        st = R_CAP;
                        break;
                    }
                }
        }
        if (!ring) {
            if (c.R.global) flags |= MF_GLOBAL;
            if (st == R_OUTSIDE) type = NT_OUTSIDE;
            else if (st == R_CAP) {
                type = NT_FAILED;
                if (lane == 0) atomicAdd(&a.diag[D_CAP], 1ull);
            } else if (st != R_OK) type = NT_FAILED;
        }
        c.neardeg = ndeg;
        if (c.neardeg) flags |= MF_NEARDEG;
        bool long_row = false;
        if (type == NT_INTERIOR) {
            int lt0 = S.find(T[0]), lt1 = S.find(T[1]), lt2 = S.find(T[2]);
            // The metadata word holds the triangle's positions in five bits.
            // In the ring order T[0] follows the whole ring of T[0]; in a
            // row longer than that a triangle vertex past the ELL width is
            // exchanged with the first entry that is not one (the order of
            // a long row's entries is its own: only this path builds it).
            auto front = [&](int& l) {
                if (l < KMAX) return;
                const int t = (lt0 != 0 && lt1 != 0 && lt2 != 0) ? 0
                            : (lt0 != 1 && lt1 != 1 && lt2 != 1) ? 1
                            : (lt0 != 2 && lt1 != 2 && lt2 != 2) ? 2 : 3;
                S.swap(l, t);
                l = t;
            };
            front(lt0);
            front(lt1);
            front(lt2);
            if (lt0 < 0 || lt1 < 0 || lt2 < 0) {
                type = NT_FAILED;
            } else {
                long_row = S.n > KMAX;
                int orow = 0;
                if (long_row) {
                    // entries KMAX.. go to an overflow row of the handle
                    int r = 0;
                    if (lane == 0) r = static_cast<int>(atomicAdd(&a.diag[D_OVF], 1ull));
                    orow = __builtin_amdgcn_readfirstlane(r);
                    if (orow >= a.out.n_ovf) {
                        type = NT_FAILED;
                        st = R_CAP;
                        if (lane == 0) atomicAdd(&a.diag[D_CAP], 1ull);
                    } else if (lane == 0) {
                        a.out.orow[slot] = orow;
                    }
                }
                if (type == NT_INTERIOR) {
                    if (lane < S.n) {
                        const uint32_t e = static_cast<uint32_t>(S.e);
                        if (lane < KMAX) {
                            a.out.idx[lane * nn + slot] = static_cast<int32_t>(e & IDX_MASK);
                            a.out.mem[lane * nn + slot] = static_cast<uint8_t>(e >> 28);
                        } else {
                            a.out.oidx[ovf_at(a.out.n_ovf, orow, lane)] = static_cast<int32_t>(e & IDX_MASK);
                            a.out.omem[ovf_at(a.out.n_ovf, orow, lane)] = static_cast<uint8_t>(e >> 28);
                        }
                    }
                    if (lane == 0) a.out.meta[slot] = meta_pack(NT_PENDING, S.n, lt0, lt1, lt2, flags);
                }
            }
        }
        if (type == NT_RING || type == NT_OUTSIDE) {
            // closure: the K nearest particles (ties by user id), picked one
            // per round as the smallest (d^2, user id) above the previous pick
            int kk = 0;
            for (int level = 0;; ++level) {
                const int hw = level < a.levels ? (sd.hw0 << level) : big;
                c.set_region(per ? make_region_periodic(sd.g, cbx, cby, hw) : make_region(sd.g, cbx, cby, hw));
                kk = 0;
                double pd = -1.0;
                int pu = -1;
                for (int r = 0; r < KNN; ++r) {
                    double bd = INFINITY;
                    int bu = INT_MAX, bt = -1;
                    c.scan([&](int t, double2 p) {
                        const double dx = p.x - q.x, dy = p.y - q.y;
                        const double d2 = dx * dx + dy * dy;
                        if (d2 < pd || d2 > bd) return;
                        const int u = c.perm[t];
                        if (d2 == pd && u <= pu) return;
                        if (d2 < bd || u < bu) {
                            bd = d2;
                            bu = u;
                            bt = t;
                        }
                    });
#pragma unroll
                    for (int m = 1; m < WAVE; m <<= 1) {
                        const double od = __shfl_xor(bd, m);
                        const int ou = __shfl_xor(bu, m), ot = __shfl_xor(bt, m);
                        if (ot >= 0 && (bt < 0 || od < bd || (od == bd && ou < bu))) {
                            bd = od;
                            bu = ou;
                            bt = ot;
                        }
                    }
                    if (bt < 0) break;
                    if (lane == 0) {
                        a.out.idx[r * nn + slot] = bt;
                        a.out.mem[r * nn + slot] = 0;
                    }
                    pd = bd;
                    pu = bu;
                    ++kk;
                }
                if (c.R.global) break;
                if (kk >= KNN && c.certify(q.x, q.y, sqrt(pd))) break;
            }
            if (c.R.global) flags |= MF_GLOBAL;
            if (kk == 0) {
                type = NT_FAILED;
            } else if (lane == 0) {
                a.out.meta[slot] = meta_pack(pending_type(type), kk, 0, 0, 0, flags);
            }
        }
        if (lane == 0) {
            if (type == NT_FAILED) {
                a.out.meta[slot] = meta_pack(NT_FAILED, 0, 0, 0, 0, flags);
                atomicAdd(&a.diag[D_FAILED], 1ull);
            }
            if (!ring) atomicAdd(&a.diag[D_ESCALATED], 1ull);
            if (flags & MF_GLOBAL) atomicAdd(&a.diag[D_GLOBAL], 1ull);
            if (c.neardeg) atomicAdd(&a.diag[D_NEARDEG], static_cast<unsigned long long>(c.neardeg));
        }
        // the row (written by several lanes) is complete before it is weighted
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (long_row) {
            // a row longer than the ELL width is solved by the wave solver
            // of k_weights_rd (one entry per lane); counted here
            if (lane == 0) {
                a.rd[atomicAdd(&a.diag[D_RDCNT], 1ull)] = static_cast<int32_t>(slot);
                atomicAdd(&a.diag[D_INTERIOR], 1ull);
                atomicMax(&a.diag[D_SUPMAX], static_cast<unsigned long long>(S.n));
            }
            continue;
        }
        // every quad of the wave computes the row's systems; they share
        // its final pass
        if constexpr (WEIGH)
            count_wave(a, weights_node<PER, WAVE / QL>(a, sd, i, j, true, slot, lane & (QL - 1), lane / QL, L.wsp,
                                                  L.wse, L.wsu, true, lane / QL));
    }
}

// The exact path's nodes, geometry and weights, one block of three waves
// per listed node (on a side stream, beside the weights pass).
template <bool PER>
__global__ void __launch_bounds__(SWG) k_slow_geom(KArgs a) {
    constexpr int WPB = SWG / WAVE;
    __shared__ int32_t svis[WPB * KROW];
    __shared__ double2 slp[WPB * STAGE];
    __shared__ int32_t slt[WPB * STAGE];
    // each ring's list (entry | ring bit << 28), its status, length and
    // near-tie count, for the ring-0 wave to merge
    __shared__ int32_t sring[WPB * KROW];
    __shared__ int sinfo[WPB * 3];
    // the weights of the finished row, by the first quad of the ring-0 wave
    __shared__ double2 wsp[(WAVE / QL) * SKP];
    __shared__ uint32_t wse[(WAVE / QL) * SKP];
    __shared__ int32_t wsu[(WAVE / QL) * SKP];
    const SlowLds L{svis, slp, slt, sring, sinfo, wsp, wse, wsu};
    slow_nodes<PER, true>(a, blockIdx.x, gridDim.x, L);
}

// Weights of the fast path's pending rows, one quad per node, nodes in the
// same 8 x 8 tiles as the fast kernel.
// One node tile of the weights pass (tile b of the build, QWG threads).
template <bool PER, class R>
__device__ __forceinline__ void weights_tile(const KArgs& a, const R& rp, int b, double2* sp, uint32_t* se,
                                             int32_t* su, int* wsum) {
    __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x & (QL - 1);
    const int qi = threadIdx.x / QL;
    const SetDesc sd = tile_set(a, b);
    int tx, ty;
    tile_xy(sd, static_cast<int>(b - sd.t0), tx, ty);
    const int i = tx * 8 + (qi & 7), j = ty * 8 + (qi >> 3);
    const bool valid = i <= sd.m.nx && j <= sd.m.ny;
    const int64_t slot = static_cast<int64_t>(b) * TILE_N + qi;
    const WaveCounts wc = weights_node<PER, 1, R>(a, sd, i, j, valid, slot, lane, qi, sp, se, su, false, 0, rp);
    // the tile's counts as one plain record, folded into the diagnostics by
    // k_weights_rd: device-wide atomics from every wave on the same few
    // counters serialise at their memory partition and stall the pass
    if (threadIdx.x % WAVE == 0) {
        for (int c = 0; c < 4; ++c) wsum[(threadIdx.x / WAVE) * TD + c] = wc.c[c];
        wsum[(threadIdx.x / WAVE) * TD + TD_KMAX] = __float_as_int(wc.kmax);
    }
    __syncthreads();
    if (threadIdx.x < TD) {
        int v = 0;
        for (int w = 0; w < QWG / WAVE; ++w) {
            const int x = wsum[w * TD + threadIdx.x];
            // (non-negative floats order as their bit patterns)
            v = (threadIdx.x == WC_SUPMAX || threadIdx.x == TD_KMAX) ? max(v, x) : v + x;
        }
        a.tdiag[static_cast<int64_t>(b) * TD + threadIdx.x] = v;
    }
}

template <bool PER, class R = StoreRows>
__global__ void __launch_bounds__(QWG) k_weights(KArgs a, R rp = R{}) {
    __shared__ double2 sp[QPB * SKP];
    __shared__ uint32_t se[QPB * SKP];
    __shared__ int32_t su[QPB * SKP];
    __shared__ int wsum[(QWG / WAVE) * TD];
    weights_tile<PER, R>(a, rp, static_cast<int>(blockIdx.x), sp, se, su, wsum);
}

// The weights pass and the exact path's geometry in one launch, on the
// caller's stream (no fork or join of a second stream): gs blocks run the
// exact path's nodes (three waves; the fourth takes part in the block's
// barriers only) and leave their rows pending, the others are the weights
// pass's tiles.  The first g1 exact-path blocks come before the tiles (the
// few nodes of an ordered cloud then start at once), the rest after them
// (the many of a sheared one, without holding back the tiles' dispatch).
// The two roles share one LDS allocation.  The exact path's rows are
// weighed after it by k_slow_weights.  With ProjRows (the fused form) the
// tiles add each finished row into its node's sum instead of storing it.
constexpr int WT_LDS = QPB * SKP * (16 + 4 + 4) + (QWG / WAVE) * BUILD_TD * 4;
constexpr int SG_LDS = 3 * KROW * 4 + 3 * STAGE * (16 + 4) + 3 * KROW * 4 + 3 * 3 * 4;
constexpr int WS_LDS = WT_LDS > SG_LDS ? WT_LDS : SG_LDS;
template <bool PER, class R = StoreRows>
__global__ void __launch_bounds__(QWG) k_weights_slow(KArgs a, int gs, int g1, int tiles, R rp = R{}) {
    __shared__ __align__(16) unsigned char lds[WS_LDS];
    const int b = static_cast<int>(blockIdx.x);
    if (b < g1 || b >= g1 + tiles) {
        double2* slp = reinterpret_cast<double2*>(lds);
        int32_t* slt = reinterpret_cast<int32_t*>(slp + 3 * STAGE);
        int32_t* svis = slt + 3 * STAGE;
        int32_t* sring = svis + 3 * KROW;
        int* sinfo = sring + 3 * KROW;
        const SlowLds L{svis, slp, slt, sring, sinfo, nullptr, nullptr, nullptr};
        slow_nodes<PER, false>(a, b < g1 ? b : b - tiles, gs, L);
        return;
    }
    double2* sp = reinterpret_cast<double2*>(lds);
    uint32_t* se = reinterpret_cast<uint32_t*>(sp + QPB * SKP);
    int32_t* su = reinterpret_cast<int32_t*>(se + QPB * SKP);
    int* wsum = su + QPB * SKP;
    weights_tile<PER, R>(a, rp, b - g1, sp, se, su, wsum);
}


// Rows listed by either weights pass because one of their systems is
// ill-conditioned (condition estimate above svd_kappa) or lost rank: every
// system of the row by the rank-revealing solver, one wave per row.  Block
// 0 first folds k_weights' per-tile counts into the diagnostics.
// The weights pass's per-tile counts folded into the diagnostics, by one
// block of QWG threads.
__device__ __forceinline__ void fold_tile_counts(const KArgs& a) {
    unsigned long long v[TD] = {0, 0, 0, 0, 0};
    const int64_t tiles = a.n_slots / TILE_N;
    for (int64_t t = threadIdx.x; t < tiles; t += QWG) {
#pragma unroll
        for (int c = 0; c < TD; ++c) {
            const unsigned long long x = static_cast<unsigned long long>(static_cast<uint32_t>(a.tdiag[t * TD + c]));
            v[c] = (c == WC_SUPMAX || c == TD_KMAX) ? max(v[c], x) : v[c] + x;
        }
    }
#pragma unroll
    for (int c = 0; c < TD; ++c)
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(v[c], off);
            v[c] = (c == WC_SUPMAX || c == TD_KMAX) ? max(v[c], o) : v[c] + o;
        }
    if (threadIdx.x % WAVE == 0) {
        if (v[WC_INTERIOR]) atomicAdd(&a.diag[D_INTERIOR], v[WC_INTERIOR]);
        if (v[WC_CLOSURE]) atomicAdd(&a.diag[D_CLOSURE], v[WC_CLOSURE]);
        if (v[WC_OUTSIDE]) atomicAdd(&a.diag[D_OUTSIDE], v[WC_OUTSIDE]);
        if (v[WC_SUPMAX]) atomicMax(&a.diag[D_SUPMAX], v[WC_SUPMAX]);
        if (v[TD_KMAX]) {
            const double k = static_cast<double>(__int_as_float(static_cast<int>(v[TD_KMAX])));
            atomicMax(&a.diag[D_GRAMCOND], static_cast<unsigned long long>(__double_as_longlong(k)));
        }
    }
}

// One row by the rank-revealing solver, by one wave, with its counts.
template <bool PER>
__device__ __forceinline__ void svd_row(const KArgs& a, int64_t slot, int lane) {
    const SetDesc sd = slot_set(a, slot);
    int i, j;
    slot_ij(sd, slot, i, j);
    int nrd = 0;
    double kmax = 0.0;
    const int nsys = wave_row_svd<PER>(a, sd, slot, node_at(sd.m, i, j, PER), lane, nrd, kmax);
    if (lane == 0) {
        atomicAdd(&a.diag[D_SVD], static_cast<unsigned long long>(nsys));
        if (nrd) atomicAdd(&a.diag[D_RANKDEF], static_cast<unsigned long long>(nrd));
        if (kmax > 0.0) atomicMax(&a.diag[D_GRAMCOND], static_cast<unsigned long long>(__double_as_longlong(kmax)));
    }
}

template <bool PER>
__global__ void __launch_bounds__(QWG) k_weights_rd(KArgs a) {
    if (blockIdx.x == 0) fold_tile_counts(a);
    const int lane = threadIdx.x & (WAVE - 1);
    const int count = static_cast<int>(a.diag[D_RDCNT]);
    const int waves = static_cast<int>(gridDim.x) * (QWG / WAVE);
    const int w0 = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x * (QWG / WAVE) + threadIdx.x / WAVE));
    for (int li = w0; li < count; li += waves) svd_row<PER>(a, a.rd[li], lane);
}

// After k_weights_slow: the exact path's rows that it left pending, weighed
// as k_slow_geom weighs them (a wave per listed node; every quad of it
// computes the row's systems and they share its final pass), a row with an
// ill-conditioned or rank-deficient system solved at once by the
// rank-revealing solver in the same wave (and listed for the adjoint,
// marked RD_SOLVED), and then the rows that the weights pass listed for
// that solver (the work of k_weights_rd: every one of them is listed
// before this launch starts, so each wave's view of the list holds them
// all, and the marked ones are skipped).  Rows longer than the ELL width
// are on that list already.  Block 0 first folds the weights pass's
// per-tile counts into the diagnostics.
template <bool PER>
__global__ void __launch_bounds__(QWG) k_slow_weights(KArgs a) {
    constexpr int WPB = QWG / WAVE;
    __shared__ double2 wsp[WPB * (WAVE / QL) * SKP];
    __shared__ uint32_t wse[WPB * (WAVE / QL) * SKP];
    __shared__ int32_t wsu[WPB * (WAVE / QL) * SKP];
    if (blockIdx.x == 0) fold_tile_counts(a);
    __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / WAVE));
    const int count = static_cast<int>(a.diag[D_SLOWCNT]);
    const int nlisted = static_cast<int>(a.diag[D_RDCNT]);
    const int waves = static_cast<int>(gridDim.x) * WPB;
    const int w0 = static_cast<int>(blockIdx.x) * WPB + wv;
    for (int li = w0; li < count; li += waves) {
        const int64_t slot = a.slow[li];
        const uint32_t meta = a.out.meta[slot];
        if (meta_type(meta) == NT_PENDING && static_cast<int>(meta_cnt(meta)) > KMAX) continue;
        const SetDesc sd = slot_set(a, slot);
        int i, j;
        slot_ij(sd, slot, i, j);
        const int o = wv * (WAVE / QL) * SKP;
        int svd = 0;
        count_wave(a, weights_node<PER, WAVE / QL>(a, sd, i, j, true, slot, lane & (QL - 1), lane / QL, wsp + o,
                                              wse + o, wsu + o, true, lane / QL, StoreRows{}, &svd));
        if (__builtin_amdgcn_readfirstlane(svd)) {
            if (lane == 0)
                a.rd[atomicAdd(&a.diag[D_RDCNT], 1ull)] = static_cast<int32_t>(static_cast<uint32_t>(slot) | RD_SOLVED);
            svd_row<PER>(a, slot, lane);
        }
    }
    for (int li = w0; li < nlisted; li += waves) {
        const int32_t e = a.rd[li];
        if (!(static_cast<uint32_t>(e) & RD_SOLVED)) svd_row<PER>(a, e, lane);
    }
}


// ------------------------------------------------ mesh-side coefficients
// The construction of App. B on the fixed mesh: for every mesh edge
// e = (a, b) of the fixed-diagonal triangulation, the minimum-norm A^m_{. e}
// solving eqs. (A0), (A1), (A2_2) over S_e = ring(a) U ring(b), ring(v) being
// v and its neighbours (i +- 1, j), (i, j +- 1), (i + 1, j + 1),
// (i - 1, j - 1) inside the mesh.  Relative to a, S_e covers ten fixed
// offsets per orientation (fewer at the mesh boundary, where the systems can
// lose rank: hence the pseudo-inverse).  Edges: horizontal (i, j)-(i+1, j)
// first, then vertical (i, j)-(i, j+1), then diagonal (i, j)-(i+1, j+1), each
// set row-major by its first end; row e of the table holds the node ids and
// coefficients of the ten offsets (coefficient 0 and node a off the mesh).
__constant__ int8_t kEdgeOff[3][MESH_SUP][2] = {
    {{-1, -1}, {-1, 0}, {0, -1}, {0, 0}, {0, 1}, {1, -1}, {1, 0}, {1, 1}, {2, 0}, {2, 1}},
    {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 0}, {0, 1}, {0, 2}, {1, 0}, {1, 1}, {1, 2}},
    {{-1, -1}, {-1, 0}, {0, -1}, {0, 0}, {0, 1}, {1, 0}, {1, 1}, {1, 2}, {2, 1}, {2, 2}}};

__global__ void __launch_bounds__(64) k_mesh_edges(MeshD m, int64_t E, int32_t* __restrict__ idx,
                                                   double* __restrict__ coef) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int64_t nh = static_cast<int64_t>(m.nx) * (m.ny + 1), nv = static_cast<int64_t>(m.nx + 1) * m.ny;
    int o, i, j;
    if (e < nh) {
        o = 0;
        i = static_cast<int>(e % m.nx);
        j = static_cast<int>(e / m.nx);
    } else if (e < nh + nv) {
        o = 1;
        i = static_cast<int>((e - nh) % (m.nx + 1));
        j = static_cast<int>((e - nh) / (m.nx + 1));
    } else {
        o = 2;
        i = static_cast<int>((e - nh - nv) % m.nx);
        j = static_cast<int>((e - nh - nv) / m.nx);
    }
    const int ib = i + (o == 1 ? 0 : 1), jb = j + (o == 0 ? 0 : 1);
    const double2 pa = node_pos(m, i, j), pb = node_pos(m, ib, jb);
    // edge frame: origin at the midpoint, unit length
    const double cx = 0.5 * (pa.x + pb.x), cy = 0.5 * (pa.y + pb.y);
    const double dxv = pa.x - pb.x, dyv = pa.y - pb.y;
    const double sc = 1.0 / sqrt(dxv * dxv + dyv * dyv);
    const double dx = dxv * sc, dy = dyv * sc;
    Moments mo;
    mo.zero();
#pragma unroll
    for (int k = 0; k < MESH_SUP; ++k) {
        const int a = i + kEdgeOff[o][k][0], b = j + kEdgeOff[o][k][1];
        if (a < 0 || b < 0 || a > m.nx || b > m.ny) continue;
        const double2 p = node_pos(m, a, b);
        mo.add((p.x - cx) * sc, (p.y - cy) * sc);
    }
    const double rhs[6] = {0.0, 0.0, 0.0, -0.5 * dx * dx, -0.5 * dx * dy, -0.5 * dy * dy};
    double y[6];
    pinv6_solve(mo, rhs, y);
#pragma unroll
    for (int k = 0; k < MESH_SUP; ++k) {
        const int a = i + kEdgeOff[o][k][0], b = j + kEdgeOff[o][k][1];
        const bool in = a >= 0 && b >= 0 && a <= m.nx && b <= m.ny;
        double c = 0.0;
        if (in) {
            const double2 p = node_pos(m, a, b);
            double pm[6];
            monos((p.x - cx) * sc, (p.y - cy) * sc, pm);
            c = dot6(pm, y);
        }
        idx[e * MESH_SUP + k] = in ? b * (m.nx + 1) + a : j * (m.nx + 1) + i;
        coef[e * MESH_SUP + k] = c;
    }
}

// Periodic box: the seam nodes (nx, j) and (i, ny) are nodes (0, j) and
// (i, 0).  The passes above skip them; their rows are copied here once the
// rows they repeat are weighted (both passes and the pseudo-inverse pass).
// A quad per node slot, in the node tiles of the other passes.
__global__ void __launch_bounds__(QWG) k_seam_copy(KArgs a) {
    const SetDesc sd = tile_set(a, blockIdx.x);
    int tx, ty;
    tile_xy(sd, static_cast<int>(blockIdx.x - sd.t0), tx, ty);
    if (tx * 8 + 7 < sd.m.nx && ty * 8 + 7 < sd.m.ny) return;  // no seam node in the tile
    const int lane = threadIdx.x & (QL - 1), qi = threadIdx.x / QL;
    const int i = tx * 8 + (qi & 7), j = ty * 8 + (qi >> 3);
    if (i > sd.m.nx || j > sd.m.ny || (i != sd.m.nx && j != sd.m.ny)) return;
    const int64_t nn = a.n_slots;
    const int64_t dst = static_cast<int64_t>(blockIdx.x) * TILE_N + (qi >> 3) * 8 + (qi & 7);
    const int64_t src = node_slot(sd, i == sd.m.nx ? 0 : i, j == sd.m.ny ? 0 : j);
    for (int k = lane; k < KMAX; k += QL) {
        a.out.idx[k * nn + dst] = a.out.idx[k * nn + src];
        a.out.mem[k * nn + dst] = a.out.mem[k * nn + src];
        a.out.w64[k * nn + dst] = a.out.w64[k * nn + src];
        if (a.out.w32) a.out.w32[k * nn + dst] = a.out.w32[k * nn + src];
    }
    if (lane == 0) {
        const uint32_t meta = a.out.meta[src];
        a.out.meta[dst] = meta;
        // a long row's overflow entries are shared, not copied
        if (row_len(meta) > KMAX) a.out.orow[dst] = a.out.orow[src];
        if (meta_type(meta) == NT_INTERIOR) atomicAdd(&a.diag[D_INTERIOR], 1ull);
        if (meta_flags(meta) & MF_RANKDEF) atomicAdd(&a.diag[D_RANKDEF], 1ull);
        if (meta_type(meta) == NT_FAILED) atomicAdd(&a.diag[D_FAILED], 1ull);
        // a copy of a row of the rank-revealing solver joins its list, which
        // the position adjoint walks (the forward is done with it)
        if (meta_flags(meta) & MF_SVD) a.rd[atomicAdd(&a.diag[D_RDCNT], 1ull)] = static_cast<int32_t>(dst);
    }
}

// The shared weights launch of the fused build, its tiles projecting, for
// the value type and channel count of the build.
template <typename TV, typename TW, typename TO>
void launch_weights_proj_t(const KArgs& a, const FusedProj& fp, int gs, int g1, int tiles, hipStream_t st) {
    const TV* v = static_cast<const TV*>(fp.vals);
    TO* o = static_cast<TO*>(fp.out);
    const unsigned grid = static_cast<unsigned>(gs + tiles);
    // (channel counts up to FUSED_CMAX: the sums stay in registers)
    switch (fp.C) {
        case 1: k_weights_slow<false, ProjRows<TV, TW, TO, 1>><<<grid, QWG, 0, st>>>(a, gs, g1, tiles, {v, o, fp.C}); break;
        case 2: k_weights_slow<false, ProjRows<TV, TW, TO, 2>><<<grid, QWG, 0, st>>>(a, gs, g1, tiles, {v, o, fp.C}); break;
        case 3: k_weights_slow<false, ProjRows<TV, TW, TO, 3>><<<grid, QWG, 0, st>>>(a, gs, g1, tiles, {v, o, fp.C}); break;
        default: k_weights_slow<false, ProjRows<TV, TW, TO, 4>><<<grid, QWG, 0, st>>>(a, gs, g1, tiles, {v, o, fp.C}); break;
    }
}
void launch_weights_proj(const KArgs& a, const FusedProj& fp, int gs, int g1, int tiles, hipStream_t st) {
    if (fp.dtype == P2M_F64) launch_weights_proj_t<double, double, double>(a, fp, gs, g1, tiles, st);
    else if (fp.dtype == P2M_F32) launch_weights_proj_t<float, float, float>(a, fp, gs, g1, tiles, st);
    else launch_weights_proj_t<uint16_t, float, float>(a, fp, gs, g1, tiles, st);
}

}  // namespace

int build_weights(const BinBuffers& b, const SetDesc* sets, int S, int64_t n_tiles, int64_t n_nodes,
                  const BuildOut& out, int levels, int fast_slots, int32_t* slow, int32_t* rd, int32_t* tdiag,
                  unsigned long long* diag, const SideWork& side, hipStream_t st, bool linear,
                  bool periodic, double svd_kappa, const FusedProj* fp) {
    PhaseTimer _timer(PH_BUILD, st);
    if (fp && (periodic || fp->C < 1 || fp->C > FUSED_CMAX)) {
        set_error("the fused build takes a bounded box and 1..%d channels", FUSED_CMAX);
        return P2M_EINVAL;
    }
    // row slots are listed as int32
    if (n_tiles * TILE_N >= (int64_t(1) << 31)) {
        set_error("too many node tiles (%lld)", static_cast<long long>(n_tiles));
        return P2M_EINVAL;
    }
    KArgs a;
    a.pos_s = reinterpret_cast<const double2*>(b.pos_s);
    a.perm = b.perm;
    a.start = b.start;
    a.sets = sets;
    a.S = S;
    a.levels = levels;
    a.n_nodes = n_nodes;
    a.n_slots = n_tiles * TILE_N;
    a.out = out;
    a.slow = slow;
    a.rd = rd;
    a.tdiag = tdiag;
    a.diag = diag;
    a.linear = linear ? 1 : 0;
    a.per = periodic ? 1 : 0;
    a.svd_kappa = svd_kappa;
    const int tiles = static_cast<int>(n_tiles);
    {
        PhaseTimer t1(PH_BUILD_FAST, st);
        // slots per lane for the expected candidate count of an interior
        // node (pi (Rf/h)^2 over four lanes, with room for fluctuation)
        if (fast_slots <= 7) k_build_fast<7><<<tiles, QWG, 0, st>>>(a);
        else if (fast_slots <= 8) k_build_fast<8><<<tiles, QWG, 0, st>>>(a);
        else k_build_fast<NS_MAX><<<tiles, QWG, 0, st>>>(a);
    }
    P2M_HIP(hipGetLastError());
    // The few nodes the fast pass could not certify take the exact wave path.
    // Its blocks loop over the actual list; their number is sized for many
    // more nodes than an ordered cloud leaves there (a sheared one leaves
    // thousands), and the blocks past the list leave at once.
    const int64_t expect = n_nodes / 64 + 64 * static_cast<int64_t>(S);
    if (!periodic) {
        // A bounded box: the exact path's geometry rides in the weights
        // pass's launch on the caller's stream (a fork and join of a second
        // stream would cost more than its rows' weights, which a short pass
        // adds after it).  The fused form's tiles project their rows; the
        // exact path's and the rank-revealing solver's rows are stored, and
        // projected after the build from the two lists.
        const int gs = static_cast<int>(std::min<int64_t>(expect, 4096));
        const int g1 = std::min(gs, 256);
        {
            PhaseTimer t3(PH_WEIGHTS, st);
            {
                PhaseTimer t4(PH_K_WEIGHTS, st);
                if (fp) launch_weights_proj(a, *fp, gs, g1, static_cast<int>(tiles), st);
                else k_weights_slow<false><<<gs + tiles, QWG, 0, st>>>(a, gs, g1, static_cast<int>(tiles));
            }
            {
                // a wave per listed row, for as many rows as the exact path
                // is sized for (a sheared cloud lists hundreds): the waves
                // past the list leave at once; the same launch takes the
                // rank-revealing solver's list
                PhaseTimer t2(PH_BUILD_SLOW, st);
                const int gw = static_cast<int>(std::min<int64_t>(std::max<int64_t>((gs + 3) / 4, 64), 1024));
                k_slow_weights<false><<<gw, QWG, 0, st>>>(a);
            }
        }
        P2M_HIP(hipGetLastError());
        return P2M_OK;
    }
    // Periodic box: the exact path on a side stream, concurrently with the
    // weights of all other nodes (without a side stream, after them on the
    // caller's stream).  (A periodic box lists hundreds of exact-path nodes,
    // whose blocks would crowd the weights pass's tiles out of a shared
    // launch.)
    const bool fork = side.stream != nullptr && side.stream != st && side.fork && side.join;
    hipStream_t sst = fork ? side.stream : st;
    if (fork) {
        P2M_HIP(hipEventRecord(side.fork, st));
        P2M_HIP(hipStreamWaitEvent(side.stream, side.fork, 0));
    }
    {
        PhaseTimer t2(PH_BUILD_SLOW, sst);
        // one block per slow node (the grid loops over the list)
        const int gs = static_cast<int>(std::min<int64_t>(expect, 4096));
        k_slow_geom<true><<<gs, SWG, 0, sst>>>(a);
    }
    P2M_HIP(hipGetLastError());
    if (fork) P2M_HIP(hipEventRecord(side.join, side.stream));
    {
        PhaseTimer t3(PH_WEIGHTS, st);
        // (one weighting code for both passes, so that a row does not depend
        // on the pass that found it)
        {
            PhaseTimer t4(PH_K_WEIGHTS, st);
            k_weights<true><<<tiles, QWG, 0, st>>>(a);
        }
        if (fork) P2M_HIP(hipStreamWaitEvent(st, side.join, 0));
        // ill-conditioned or rank-deficient rows of either pass (normally none)
        // (a wave per listed row; the grid loops over the list)
        {
            PhaseTimer t5(PH_K_WEIGHTS_RD, st);
            k_weights_rd<true><<<64, QWG, 0, st>>>(a);
        }
        k_seam_copy<<<tiles, QWG, 0, st>>>(a);
    }
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

int64_t mesh_edge_count(const MeshD& m) {
    return static_cast<int64_t>(m.nx) * (m.ny + 1) + static_cast<int64_t>(m.nx + 1) * m.ny +
           static_cast<int64_t>(m.nx) * m.ny;
}

int mesh_edge_table(const MeshD& m, int32_t* idx, double* coef, hipStream_t st) {
    const int64_t E = mesh_edge_count(m);
    k_mesh_edges<<<static_cast<unsigned>((E + 63) / 64), 64, 0, st>>>(m, E, idx, coef);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
