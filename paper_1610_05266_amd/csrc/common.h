// Internal definitions shared by the HIP translation units of libp2m.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "p2m.h"

namespace p2m {

// Uniform mesh as the kernels see it.
struct MeshD {
    int nx, ny;
    double H, x0, y0;
};

// Binning grid: kb x kb square bins per mesh cell, bins cover the mesh
// rectangle exactly; bin (bx, by) has key by*nbx + bx.  Key nbins collects
// particles that are outside the mesh or non-finite (excluded everywhere).
struct Grid {
    int nbx, nby, kb;
    double bw, x0, y0;
};

// Diagnostics counters (device int64 array, one build).
enum DiagIdx : int {
    D_INTERIOR = 0,
    D_CLOSURE,
    D_OUTSIDE,
    D_RANKDEF,
    D_CAP,
    D_ESCALATED,
    D_GLOBAL,
    D_NEARDEG,
    D_BAD,
    D_FAILED,
    D_SUPMAX,
    D_DUP,
    D_SLOWCNT,  // length of the slow-path node list
    D_RDCNT,    // length of the list of rows for the rank-revealing solver
    D_SVD,      // moment systems solved by the rank-revealing solver
    D_GRAMCOND, // largest condition number of a full-rank system's Gram
                // matrix (bits of a non-negative double: ordered as integers)
    D_BWDSKIP,  // rank-deficient systems the last position adjoint left out
    D_OVF,      // rows longer than KMAX (overflow rows taken)
    D_COUNT
};

// An entry of the rank-revealing solver's row list with this bit set names a
// row solved that way already (listed for the adjoint, which also reads the
// list).
constexpr uint32_t RD_SOLVED = 0x80000000u;

// A row holds up to KROW support entries: the first KMAX in the ELL arrays
// of its node slot, the rest (rows found by the exact path around vertices of
// high degree, rare) in an overflow row of the same layout, whose index is
// kept per slot.
constexpr int KMAX = 32;               // ELL entries stored per node slot
constexpr int KROW = P2M_MAX_SUPPORT;  // longest row (count field: 6 bits)
static_assert(KROW <= 63 && KROW > KMAX, "row count fits the metadata word");
constexpr int KNN = P2M_CLOSURE_K;
constexpr int CMAX = 16;  // channels per call (checked at the boundary)

// Per-node metadata word of the ELL weights.
// NT_PENDING*: node whose support is known (interior: ring union; closure:
// nearest particles, ring or outside-hull) but whose weights are still to be
// computed (transient inside one build).
enum NodeType : uint32_t {
    NT_INTERIOR = 0, NT_RING = 1, NT_OUTSIDE = 2, NT_FAILED = 3,
    NT_PENDING = 4, NT_PEND_RING = 5, NT_PEND_OUT = 6
};
// bits 0-2 type, 3-8 count, 9-13 / 14-18 / 19-23 ELL slots of the triangle's
// vertices, 24- flags
__host__ __device__ inline uint32_t meta_pack(uint32_t type, uint32_t cnt, uint32_t ta, uint32_t tb,
                                              uint32_t tc, uint32_t flags) {
    return type | (cnt << 3) | (ta << 9) | (tb << 14) | (tc << 19) | (flags << 24);
}
__host__ __device__ inline uint32_t meta_type(uint32_t m) { return m & 7u; }
__host__ __device__ inline uint32_t meta_cnt(uint32_t m) { return (m >> 3) & 63u; }
// Row length for readers of finished rows: never beyond KROW.
__host__ __device__ inline int row_len(uint32_t m) {
    const int n = static_cast<int>((m >> 3) & 63u);
    return n < KROW ? n : KROW;
}
__host__ __device__ inline uint32_t meta_t(uint32_t m, int k) { return (m >> (9 + 5 * k)) & 31u; }
constexpr uint32_t MF_NEARDEG = 1u, MF_RANKDEF = 2u, MF_ESCALATED = 4u, MF_GLOBAL = 8u;
// MF_SVD: the row's systems were solved by the rank-revealing solver;
// MF_RD0 << e: system e of the row (the closure's one system: e = 0) has
// rank below 6 (its weights are the minimum-norm least-squares answer).
constexpr uint32_t MF_SVD = 16u, MF_RD0 = 32u;
__host__ __device__ inline uint32_t meta_flags(uint32_t m) { return m >> 24; }

// Membership bits stored per ELL entry: bit k set when the particle belongs to
// the Delaunay ring of the k-th vertex of the node's triangle.
constexpr uint8_t MB_RING_A = 1, MB_RING_B = 2, MB_RING_C = 4;

// One particle set of a batch: its own mesh, binning grid and fast-path
// radii, and where its particles, nodes, bins and node tiles start in the
// concatenated arrays.  A single-set build is a batch of one.
struct SetDesc {
    MeshD m;
    Grid g;
    int64_t p0;       // first particle (user order)
    int64_t n0;       // first mesh node
    int64_t b0;       // first bin
    int64_t t0;       // first 8 x 8 node tile
    int32_t tiles_x;  // node tiles per row
    int32_t hw0;      // slow path: half-width (bins) of the first region
    int32_t hwf;      // fast path: half-width (bins) scanned for interior nodes
    int32_t hwc;      // fast path: half-width (bins) scanned for ring nodes
    double Rf;        // fast path: candidate radius of interior nodes
    double Rc;        // fast path: candidate radius of boundary-ring nodes
    double h;         // the caller's particle spacing: the length unit of a
                      // closure system solved by the rank-revealing solver
};

// Index of the set that holds item v, where first(s) is the first item of
// set s (non-decreasing in s).  Uniform loads; S = 1 costs nothing.
template <class F>
__device__ __forceinline__ int set_search(int S, int64_t v, F&& first) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---- node slots of the ELL rows
// Rows are stored per node slot rather than per mesh node: node (i, j) of
// node tile t (8 x 8 nodes) has slot 64 t + 8 (j % 8) + (i % 8), with tiles
// numbered as the build launches take them (tile_xy).  The 64 nodes of a
// tile, and the 16 nodes of a wave, occupy consecutive slots, so one entry
// of a wave's rows is a single aligned 128-byte FP64 segment.  Slots of a
// partial tile that lie beyond the mesh hold empty rows.
constexpr int TILE_N = 64;

// Tile tl of a set's node tiles: the full tiles first (by rows, each row
// rotated by its index), then the
// partial tiles of the last column and of the last row.  The hardware
// dispatches blocks in index order and holds a fixed number at a time, so
// full tiles taken in whole rounds, with the cheap partial ones filling the
// last slots, finish earlier than the row-major order.
__host__ __device__ inline void tile_xy(const SetDesc& sd, int tl, int& tx, int& ty) {
    const int fx = (sd.m.nx + 1) / 8, fy = (sd.m.ny + 1) / 8;  // full tile columns, rows
    if (tl < fx * fy) {
        // rows of full tiles rotated by their row index: consecutive blocks
        // go to the eight XCDs in turn, and the tiles of one mesh column
        // (the heavier edge columns among them) are spread over all XCDs
        // instead of sharing one when fx is a multiple of eight
        ty = tl / fx;
        tx = (tl % fx + ty) % fx;
        return;
    }
    int r = tl - fx * fy;
    if (sd.tiles_x > fx) {
        if (r < fy) {
            tx = fx;
            ty = r;
            return;
        }
        r -= fy;
    }
    tx = r;
    ty = fy;
}
// Inverse of tile_xy.
__host__ __device__ inline int tile_index(const SetDesc& sd, int tx, int ty) {
    const int fx = (sd.m.nx + 1) / 8, fy = (sd.m.ny + 1) / 8;
    if (tx < fx && ty < fy) return ty * fx + (tx - ty % fx + fx) % fx;
    if (ty < fy) return fx * fy + ty;                  // the partial column
    return fx * fy + (sd.tiles_x > fx ? fy : 0) + tx;  // the partial row
}
__host__ __device__ inline int64_t node_slot(const SetDesc& sd, int i, int j) {
    return (sd.t0 + tile_index(sd, i >> 3, j >> 3)) * TILE_N + (j & 7) * 8 + (i & 7);
}
// Node (i, j) of a slot of set sd (the slot's tile must belong to sd); false
// beyond the mesh.
__host__ __device__ inline bool slot_ij(const SetDesc& sd, int64_t slot, int& i, int& j) {
    int tx, ty;
    tile_xy(sd, static_cast<int>(slot / TILE_N - sd.t0), tx, ty);
    const int l = static_cast<int>(slot % TILE_N);
    i = tx * 8 + (l & 7);
    j = ty * 8 + (l >> 3);
    return i <= sd.m.nx && j <= sd.m.ny;
}
__host__ __device__ inline int64_t ij_node(const SetDesc& sd, int i, int j) {
    return sd.n0 + static_cast<int64_t>(j) * (sd.m.nx + 1) + i;
}

// Everything the kernels need to know about one weights handle.
struct WeightsView {
    const SetDesc* sets;    // [S] device
    int S;
    int64_t n_nodes;        // all sets
    int64_t n_slots;        // node slots of all sets (64 per node tile)
    int64_t N;              // all sets
    const uint32_t* meta;   // [n_slots]
    const int32_t* idx;     // [KMAX][n_slots] user particle ids
    const double* w64;      // [KMAX][n_slots]
    const float* w32;       // [KMAX][n_slots] or null
    const uint8_t* mem;     // [KMAX][n_slots]
    const int32_t* orow;    // [n_slots] overflow row of a slot (rows longer than KMAX only)
    const int32_t* oidx;    // [KROW - KMAX][n_ovf] entries KMAX.. of overflow rows
    const double* ow64;
    const float* ow32;
    const uint8_t* omem;
    int64_t n_ovf;          // overflow rows (capacity)
    const int32_t* rd;      // row slots solved by the rank-revealing solver
    unsigned long long* diag;  // the build's diagnostics (count of rd: D_RDCNT)
    const double2* pos_s;   // [N] positions in bin order (the binning)
    const int32_t* perm;    // [N] bin order -> user id
    const int32_t* start;   // first bin-order slot of every bin (bins of set s from sets[s].b0)
    // Particle-major index of the entries (handles built with
    // P2M_DETERMINISTIC, else null): the entries that reference user
    // particle u are tent[tptr[u] .. tptr[u + 1]), ascending, each an entry
    // index (see entry_at) with its node in tnode; gent is per-entry scratch
    // of the position adjoint.
    const int32_t* tptr;    // [N + 1]
    const int32_t* tent;
    const int32_t* tnode;
    double2* gent;          // [n_ent]
};

// Entry index of entry k of slot s: k * n_slots + s in the ELL arrays, else
// KMAX * n_slots + its overflow index (n_ent = KMAX n_slots + (KROW - KMAX) n_ovf).
__host__ __device__ inline int64_t entry_at(int64_t n_slots, int64_t n_ovf, int32_t orow, int64_t s, int k) {
    return k < KMAX ? static_cast<int64_t>(k) * n_slots + s
                    : KMAX * n_slots + static_cast<int64_t>(k - KMAX) * n_ovf + orow;
}

// Index of entry k (>= KMAX) of an overflow row r in the overflow arrays.
__host__ __device__ inline int64_t ovf_at(int64_t n_ovf, int32_t r, int k) {
    return static_cast<int64_t>(k - KMAX) * n_ovf + r;
}

// Exact-rounding helpers: products/sums that must not be contracted into
// FMAs (node coordinates are defined as x0 + i*H with two roundings).
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }

// Position of mesh node (i, j): (x0 + i H, y0 + j H), each coordinate rounded
// twice (product, then sum), never fused.
__device__ __forceinline__ double2 node_pos(const MeshD& m, int i, int j) {
    return make_double2(add_rn(m.x0, mul_rn(static_cast<double>(i), m.H)),
                        add_rn(m.y0, mul_rn(static_cast<double>(j), m.H)));
}

// ------------------------------------------------------------ periodic box
// With the periodic option the box [x0, x0 + nx H) x [y0, y0 + ny H) is a
// torus: a particle enters every computation of a node as its image nearest
// to the node (position plus a multiple of the period, one rounding per
// coordinate), and node (nx, j) / (i, ny) is node (0, j) / (i, 0).
__device__ __forceinline__ double2 image_near(const MeshD& m, double2 p, double2 q) {
    const double Lx = mul_rn(static_cast<double>(m.nx), m.H), Ly = mul_rn(static_cast<double>(m.ny), m.H);
    const double kx = rint((q.x - p.x) / Lx), ky = rint((q.y - p.y) / Ly);
    return make_double2(add_rn(p.x, mul_rn(kx, Lx)), add_rn(p.y, mul_rn(ky, Ly)));
}
__device__ __forceinline__ double2 node_at(const MeshD& m, int i, int j, bool per) {
    return per ? node_pos(m, i == m.nx ? 0 : i, j == m.ny ? 0 : j) : node_pos(m, i, j);
}

// Value of v in lane (lane ^ m) of the same group of W lanes (m < W).  For
// quads the exchange is a DPP quad permute ([1,0,3,2] for m = 1, [2,3,0,1]
// for m = 2, [3,2,1,0] for m = 3) that needs no LDS round trip; the four
// lanes must be active.  A quad permute always reads a lane of its own quad,
// so every lane is written and the destination needs no prior value
// (bound_ctrl set).
template <int W>
__device__ __forceinline__ int lane_xor(int v, int m) {
    if constexpr (W == 4) {
        return m == 1   ? __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true)
               : m == 2 ? __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true)
                        : __builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, true);
    } else {
        return __shfl_xor(v, m, W);
    }
}
template <int W>
__device__ __forceinline__ double lane_xor(double v, int m) {
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor<W>(static_cast<int>(b), m);
    const int hi = lane_xor<W>(static_cast<int>(b >> 32), m);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <int W>
__device__ __forceinline__ float lane_xor(float v, int m) {
    return __int_as_float(lane_xor<W>(__float_as_int(v), m));
}

// Field element loads/stores with widening to the accumulation type.
__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
    return __uint_as_float(static_cast<uint32_t>(v) << 16);
}
// Field element load widened to the accumulation type.
__device__ __forceinline__ double ld(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ld(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ld(const uint16_t* p, int64_t i) { return bf16_to_f32(p[i]); }

// One node's weighted sum of eq. (p2m) by the four lanes of a quad: lane l
// adds the entries k = l, l + 4, ... in ascending k (add), then the partial
// sums are combined in a fixed order and lane c % 4 stores channel c
// (store).  The stored-weights projection and the fused build share it, so
// both give the same bits.
template <typename TV, typename TW, typename TO, int CC>
struct RowSum {
    static constexpr int NC = CC > 0 ? CC : CMAX;
    TW acc[NC];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = TW(0);
    }
    __device__ __forceinline__ void add(TW wk, const TV* vals, int64_t j, int C) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < C) acc[c] += wk * static_cast<TW>(ld(vals, j * C + c));
    }
    __device__ __forceinline__ void store(TO* out, int64_t node, int C, int lane) {
        // (a constant trip count: the loop unrolls and acc stays in registers)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c < C) {
                TW v = acc[c];
                v += lane_xor<4>(v, 1);
                v += lane_xor<4>(v, 2);
                if (lane == (c & 3)) out[node * C + c] = static_cast<TO>(v);
            }
        }
    }
};

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

}  // namespace p2m

// Host-side launch helpers (defined in capi.hip).
namespace p2m {
void set_error(const char* fmt, ...);
int hip_check(hipError_t e, const char* what);
}  // namespace p2m

#define P2M_HIP(call)                                              \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return ::p2m::hip_check(_e, #call);  \
    } while (0)
