// C ABI of libp2m: argument validation, handle and workspace management,
// diagnostics and error reporting.  All device work is in the other files.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

namespace p2m {

namespace {
thread_local std::string g_err = "no error";

constexpr int NS_FAST_MAX = 10;  // candidate slots per lane of the fast pass, at most

// Process-wide tuning knobs (set with p2m_set_option).
struct Tuning {
    double bin_scale = 1.0;       // bin width ~ bin_scale * h
    double region_h = 4.0;        // slow path: first search half-width, in units of h
    double fast_radius = 2.6;     // fast path: candidate radius, in units of h
    double closure_radius = 4.0;  // fast path, boundary ring: candidate radius / h
    int levels = 3;               // doublings before the global scan
    // condition estimate trace(G) trace(G^-1) above which a moment system
    // goes to the rank-revealing solver: 1e8 keeps Cholesky (with one
    // refinement step) within about eps cond(M) of the minimum-norm answer
    double svd_cond = 1e8;
    int m2p_ppt = 1;  // particles per thread of the M2P kernel (1, 2 or 4)
} g_tune;

// Candidate slots per lane for pi (Rf/h)^2 expected candidates, with a margin
// for the fluctuation of the count: 7 up to 21.5 (Rf <= ~2.6h), 8 up to 26
// (~2.9h), else 10.  Every slot is evaluated in every gift-wrapping step.
int fast_slots() {
    const double expect = 3.14159265358979 * g_tune.fast_radius * g_tune.fast_radius;
    return expect <= 21.5 ? 7 : (expect <= 26.0 ? 8 : NS_FAST_MAX);
}
}  // namespace

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

int hip_check(hipError_t e, const char* what) {
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? P2M_ENOMEM : P2M_EHIP;
}

// Sizes of all sets of a batch together.
struct SetTotals {
    int64_t N = 0, n_nodes = 0, nbins = 0, n_tiles = 0;
};

// ---------------------------------------------------- static workspace
// The workspace of p2m_project_fused_noalloc: a file-scope device array, of
// which every GPU the library runs on holds its own copy until the process
// ends.  Its name in host code is a host-side stand-in: host code takes the
// array's device address once per device (hipGetSymbolAddress, with that
// device current) and uses only that address, carving the build's buffers
// from it.
constexpr int64_t NA_MAX_N = int64_t(1) << 17;     // particles
constexpr int64_t NA_MAX_TILES = 256;              // 8 x 8 node tiles (e.g. 127 x 127 cells)
constexpr int64_t NA_MAX_SLOTS = NA_MAX_TILES * TILE_N;
constexpr int64_t NA_MAX_BINS = int64_t(1) << 18;  // binning grid
constexpr int64_t NA_MAX_HIST = 16384;             // (super-bin, chunk) counters
constexpr int64_t NA_MAX_TSUM = 1024;              // scan tiles of those
constexpr int64_t NA_OVF = 256;                    // rows longer than the ELL width
constexpr size_t na_align(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Byte offsets of the buffers in the array (each 256-byte aligned).
struct NaLayout {
    size_t key, rank, perm, pos_s, part_pos, part_key, part_uid, start, hist, tsum;
    size_t meta, slow, rd, tdiag, idx, w64, w32, mem, orow, oidx, ow64, ow32, omem, diag, sets, total;
};
constexpr NaLayout na_layout() {
    NaLayout L{};
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o += na_align(bytes);
        return at;
    };
    L.key = take(4 * NA_MAX_N);
    L.rank = take(4 * NA_MAX_N);
    L.perm = take(4 * NA_MAX_N);
    L.pos_s = take(16 * NA_MAX_N);
    L.part_pos = take(16 * NA_MAX_N);
    L.part_key = take(4 * NA_MAX_N);
    L.part_uid = take(4 * NA_MAX_N);
    L.start = take(4 * (NA_MAX_BINS + 2));
    L.hist = take(4 * (NA_MAX_HIST + 1));
    L.tsum = take(4 * (NA_MAX_TSUM + 1));
    L.meta = take(4 * NA_MAX_SLOTS);
    L.slow = take(4 * NA_MAX_SLOTS);
    L.rd = take(4 * NA_MAX_SLOTS);
    L.tdiag = take(4 * BUILD_TD * NA_MAX_TILES);
    L.idx = take(4 * KMAX * NA_MAX_SLOTS);
    L.w64 = take(8 * KMAX * NA_MAX_SLOTS);
    L.w32 = take(4 * KMAX * NA_MAX_SLOTS);
    L.mem = take(1 * KMAX * NA_MAX_SLOTS);
    L.orow = take(4 * NA_MAX_SLOTS);
    L.oidx = take(4 * (KROW - KMAX) * NA_OVF);
    L.ow64 = take(8 * (KROW - KMAX) * NA_OVF);
    L.ow32 = take(4 * (KROW - KMAX) * NA_OVF);
    L.omem = take(1 * (KROW - KMAX) * NA_OVF);
    L.diag = take(8 * D_COUNT);
    L.sets = take(sizeof(SetDesc));
    L.total = o;
    return L;
}
constexpr NaLayout NA = na_layout();

}  // namespace p2m

// The static workspace of p2m_project_fused_noalloc (layout: na_layout).
static __device__ __align__(256) unsigned char scratch[p2m::NA.total];

using namespace p2m;

struct p2m_weights {
    int device = -1;
    int S = 0;                        // particle sets (1 unless built from a batch)
    std::vector<p2m::SetDesc> hsets;  // host copy of the device set table
    p2m::SetDesc* dsets = nullptr;    // device set table [capSets]
    int64_t N = 0;
    int64_t n_nodes = 0;
    int64_t n_tiles = 0;
    int flags = 0;
    // capacities of the device buffers
    int64_t capN = 0, capBins = 0, capNodes = 0, capSlots = 0, capTiles = 0, capSets = 0, capHist = 0;
    // slots the FP32 weights hold: tracked on their own, since a build
    // without P2M_WEIGHTS_F32 grows the other row buffers but not these
    int64_t capSlots32 = 0;
    BinBuffers bins{};
    uint32_t* meta = nullptr;  // ELL rows per node slot (64 per node tile)
    int32_t* idx = nullptr;
    int32_t* slow = nullptr;
    int32_t* rd = nullptr;
    int32_t* tdiag = nullptr;  // per node tile records of the weights pass [BUILD_TD per tile]
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;  // side-stream fork / join
    double* w64 = nullptr;
    float* w32 = nullptr;
    uint8_t* mem = nullptr;
    // rows longer than the ELL width: overflow row per slot, and the
    // overflow rows' entries KMAX.. ([KROW - KMAX][capOvf] each)
    int32_t* orow = nullptr;
    int32_t* oidx = nullptr;
    double* ow64 = nullptr;
    float* ow32 = nullptr;
    uint8_t* omem = nullptr;
    int64_t capOvf = 0, capOvf32 = 0;
    // particle-major index of the entries (P2M_DETERMINISTIC): counts or
    // cursors [N], range starts [N + 1], entry indices and their nodes
    // [n_ent], scan tile totals, and the per-entry position adjoint [n_ent]
    int32_t* tcnt = nullptr;
    int32_t* tptr = nullptr;
    int32_t* tent = nullptr;
    int32_t* tnode = nullptr;
    int32_t* ttile = nullptr;
    double2* gent = nullptr;
    int64_t capTN = 0, capTE = 0, capTT = 0;
    // the last build projected its values as it weighted them and kept the
    // weights of the exact and rank-revealing rows only (p2m_project_fused)
    bool rows_only = false;
    unsigned long long* diag = nullptr;
};

struct p2m_batch {
    int device = -1;
    std::vector<p2m_mesh> meshes;
    std::vector<double> h;
    std::vector<int64_t> off;            // [S + 1] particle offsets
    std::vector<p2m::SetDesc> sets;      // host copy of the device table
    p2m::SetTotals tot;
    p2m::SetDesc* dsets = nullptr;       // device [S], for the batched M2P
    int S() const { return static_cast<int>(meshes.size()); }
};

// Mesh-side quadratically consistent functions: the edge table of one mesh.
struct p2m_mesh_qcsf {
    p2m::MeshD m{};
    int64_t E = 0;
    int32_t* idx = nullptr;  // [E][MESH_SUP] support node ids
    double* coef = nullptr;  // [E][MESH_SUP] coefficients A^m
    bool per = false;        // periodic box: every edge takes its interior coefficients
};

namespace {

template <typename T>
int grow(T** p, int64_t count, int64_t have) {
    if (*p && have >= count) return P2M_OK;
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * static_cast<size_t>(count));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_check(e, "hipMalloc");
    }
    return P2M_OK;
}

void release(p2m_weights* w) {
    void* ptrs[] = {w->bins.key, w->bins.rank, w->bins.hist, w->bins.start, w->bins.tsum, w->bins.pos_s,
                    w->bins.perm, w->bins.part_pos, w->bins.part_key, w->bins.part_uid, w->meta, w->idx, w->slow,
                    w->rd, w->tdiag, w->w64, w->w32, w->mem, w->diag, w->dsets, w->orow, w->oidx, w->ow64,
                    w->ow32, w->omem, w->tcnt, w->tptr, w->tent, w->tnode, w->ttile, w->gent};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (w->ev_fork) (void)hipEventDestroy(w->ev_fork);
    if (w->ev_join) (void)hipEventDestroy(w->ev_join);
}

bool is_fin(double v) { return std::isfinite(v); }

int check_mesh(const p2m_mesh* m) {
    if (!m) {
        set_error("mesh is NULL");
        return P2M_EINVAL;
    }
    if (m->nx < 1 || m->ny < 1 || !(m->H > 0.0) || !is_fin(m->H) || !is_fin(m->x0) || !is_fin(m->y0)) {
        set_error("invalid mesh (nx=%d ny=%d H=%g)", m->nx, m->ny, m->H);
        return P2M_EINVAL;
    }
    const int64_t nn = static_cast<int64_t>(m->nx + 1) * (m->ny + 1);
    if (nn * KMAX >= (int64_t(1) << 40)) {
        set_error("mesh too large");
        return P2M_EINVAL;
    }
    return P2M_OK;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t dsize(int dtype) { return dtype == P2M_F64 ? 8 : dtype == P2M_F32 ? 4 : 2; }

int check_vals(const void* p, int C, int dtype, const char* what, bool mesh_side) {
    if (C < 1 || C > CMAX) {
        set_error("C=%d out of range [1, 16]", C);
        return P2M_EINVAL;
    }
    if (dtype != P2M_F64 && dtype != P2M_F32 && dtype != P2M_BF16) {
        set_error("unknown dtype %d", dtype);
        return P2M_EINVAL;
    }
    if (!p) {
        set_error("%s is NULL", what);
        return P2M_EINVAL;
    }
    const size_t a = mesh_side && dtype == P2M_BF16 ? 4 : dsize(dtype);
    if (!aligned(p, a)) {
        set_error("%s is misaligned", what);
        return P2M_EINVAL;
    }
    return P2M_OK;
}

MeshD to_meshd(const p2m_mesh* m) { return MeshD{m->nx, m->ny, m->H, m->x0, m->y0}; }

WeightsView view(const p2m_weights* w) {
    WeightsView v;
    v.sets = w->dsets;
    v.S = w->S;
    v.n_nodes = w->n_nodes;
    v.n_slots = w->n_tiles * TILE_N;
    v.N = w->N;
    v.meta = w->meta;
    v.idx = w->idx;
    v.w64 = w->w64;
    v.w32 = (w->flags & P2M_WEIGHTS_F32) ? w->w32 : nullptr;
    v.mem = w->mem;
    v.orow = w->orow;
    v.oidx = w->oidx;
    v.ow64 = w->ow64;
    v.ow32 = (w->flags & P2M_WEIGHTS_F32) ? w->ow32 : nullptr;
    v.omem = w->omem;
    v.n_ovf = w->capOvf;
    v.rd = w->rd;
    v.diag = w->diag;
    v.pos_s = reinterpret_cast<const double2*>(w->bins.pos_s);
    v.perm = w->bins.perm;
    v.start = w->bins.start;
    const bool det = (w->flags & P2M_DETERMINISTIC) != 0;
    v.tptr = det ? w->tptr : nullptr;
    v.tent = det ? w->tent : nullptr;
    v.tnode = det ? w->tnode : nullptr;
    v.gent = det ? w->gent : nullptr;
    return v;
}

int check_handle(const p2m_weights* w) {
    if (!w || w->n_nodes <= 0) {
        set_error("weights handle is NULL or was never built");
        return P2M_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != w->device) {
        set_error("weights handle belongs to device %d, current device is %d", w->device, dev);
        return P2M_EINVAL;
    }
    return P2M_OK;
}

// A handle whose rows hold weights (not the workspace of a fused projection).
int check_rows(const p2m_weights* w) {
    int rc = check_handle(w);
    if (!rc && w->rows_only) {
        set_error("the last build of this handle was a fused projection, which keeps no weights");
        rc = P2M_EINVAL;
    }
    return rc;
}

// Set table of a batch: grid, fast-path radii and offsets of every set from
// its mesh, its particle spacing h and the current tuning options.
int make_sets(const p2m_mesh* meshes, const double* hs, const int64_t* off, int S, std::vector<SetDesc>& sets,
              SetTotals& tot) {
    sets.assign(S, SetDesc{});
    tot = SetTotals{};
    if (off[0] != 0) {
        set_error("set_offsets[0] must be 0");
        return P2M_EINVAL;
    }
    for (int s = 0; s < S; ++s) {
        int rc = check_mesh(&meshes[s]);
        if (rc) return rc;
        const p2m_mesh& mesh = meshes[s];
        const double h = hs[s];
        if (!(h > 0.0) || !is_fin(h)) {
            set_error("set %d: h must be positive and finite (got %g)", s, h);
            return P2M_EINVAL;
        }
        const int64_t Ns = off[s + 1] - off[s];
        if (Ns < 3) {
            set_error("set %d has %lld particles (at least 3 needed)", s, static_cast<long long>(Ns));
            return P2M_EINVAL;
        }
        // binning grid: kb x kb bins per cell, bin width close to bin_scale * h
        const double want = g_tune.bin_scale * h;
        int64_t kb = std::max<int64_t>(1, std::llround(mesh.H / want));
        while (kb > 1 && static_cast<double>(mesh.nx) * kb * static_cast<double>(mesh.ny) * kb > 1.0e9) --kb;
        SetDesc& d = sets[s];
        d.m = to_meshd(&mesh);
        d.g.kb = static_cast<int>(kb);
        d.g.nbx = static_cast<int>(mesh.nx * kb);
        d.g.nby = static_cast<int>(mesh.ny * kb);
        d.g.bw = mesh.H / static_cast<double>(kb);
        d.g.x0 = mesh.x0;
        d.g.y0 = mesh.y0;
        d.p0 = off[s];
        d.n0 = tot.n_nodes;
        d.b0 = tot.nbins;
        d.t0 = tot.n_tiles;
        d.tiles_x = (mesh.nx + 1 + 7) / 8;
        d.hw0 = std::max(2, static_cast<int>(std::ceil(g_tune.region_h * h / d.g.bw)));
        d.Rf = g_tune.fast_radius * h;
        d.hwf = std::max(1, static_cast<int>(std::ceil(d.Rf / d.g.bw)));
        d.Rc = g_tune.closure_radius * h;
        d.h = h;
        d.hwc = std::max(1, static_cast<int>(std::ceil(d.Rc / d.g.bw)));
        tot.n_nodes += static_cast<int64_t>(mesh.nx + 1) * (mesh.ny + 1);
        tot.nbins += static_cast<int64_t>(d.g.nbx) * d.g.nby;
        tot.n_tiles += static_cast<int64_t>(d.tiles_x) * ((mesh.ny + 1 + 7) / 8);
    }
    tot.N = off[S];
    if (tot.N >= (int64_t(1) << 28)) {
        set_error("N=%lld particles in all sets, at most 2^28 - 1", static_cast<long long>(tot.N));
        return P2M_EINVAL;
    }
    if (tot.nbins >= (int64_t(1) << 31) - 2) {
        set_error("binning grid too large (%lld bins)", static_cast<long long>(tot.nbins));
        return P2M_EINVAL;
    }
    // row slots (64 per node tile) are listed as int32
    if (tot.n_nodes * KMAX >= (int64_t(1) << 40) || tot.n_tiles * TILE_N >= (int64_t(1) << 31)) {
        set_error("meshes too large (%lld nodes)", static_cast<long long>(tot.n_nodes));
        return P2M_EINVAL;
    }
    return P2M_OK;
}

// Shared by the single-set and batched builds: workspace, set table upload
// (only when it changed), binning and the three build kernels.
// Arguments of a build that do not depend on the workspace.
int check_build(const std::vector<SetDesc>& sets, const double* pos, int flags) {
    if (!pos || !aligned(pos, 16)) {
        set_error("pos is NULL or not 16-byte aligned");
        return P2M_EINVAL;
    }
    if (flags & ~(P2M_WEIGHTS_F32 | P2M_STRICT | P2M_LINEAR | P2M_PERIODIC | P2M_DETERMINISTIC)) {
        set_error("unknown flags 0x%x", flags);
        return P2M_EINVAL;
    }
    if (flags & P2M_PERIODIC)
        for (const SetDesc& d : sets)
            if (d.m.nx < 4 || d.m.ny < 4) {
                set_error("a periodic box needs at least 4 cells per side (nx=%d ny=%d)", d.m.nx, d.m.ny);
                return P2M_EINVAL;
            }
    return P2M_OK;
}

// The build's launches on a handle whose buffers and device set table are
// in place: binning, then the build kernels (slow path on side.stream, or on
// st when side.stream is null).
int launch_build(p2m_weights* w, const SetTotals& tot, const double* pos, int flags, const SideWork& side,
                 hipStream_t st, const FusedProj* fp = nullptr) {
    w->rows_only = fp != nullptr;
    // (the binning clears the diagnostics before anything counts into them)
    int rc = bin_particles(w->bins, pos, tot.N, w->dsets, w->S, tot.nbins, w->diag, st);
    if (rc) return rc;
    const bool want32 = (flags & P2M_WEIGHTS_F32) != 0;
    BuildOut out{w->meta, w->idx, w->w64, want32 ? w->w32 : nullptr, w->mem,
                 w->orow, w->oidx, w->ow64, want32 ? w->ow32 : nullptr, w->omem, w->capOvf};
    rc = build_weights(w->bins, w->dsets, w->S, tot.n_tiles, tot.n_nodes, out, g_tune.levels, fast_slots(),
                       w->slow, w->rd, w->tdiag, w->diag, side, st, (flags & P2M_LINEAR) != 0,
                       (flags & P2M_PERIODIC) != 0, g_tune.svd_cond, fp);
    if (!rc && (flags & P2M_DETERMINISTIC))
        rc = build_transpose(view(w), w->tcnt, w->tptr, w->tent, w->tnode, w->ttile, st);
    return rc;
}

int build_sets(const std::vector<SetDesc>& sets, const SetTotals& tot, const double* pos, int flags,
               p2m_weights** wout, hipStream_t st, const FusedProj* fp = nullptr) {
    int rc0 = check_build(sets, pos, flags);
    if (rc0) return rc0;
    if (!wout) {
        set_error("output handle pointer is NULL");
        return P2M_EINVAL;
    }
    int nch = 0, sbs = 0, nsb = 0;
    int rc = bin_layout(tot.N, tot.nbins, &nch, &sbs, &nsb);
    if (rc) return rc;
    int dev = 0;
    P2M_HIP(hipGetDevice(&dev));
    p2m_weights* w = *wout;
    bool fresh = false;
    if (!w) {
        w = new (std::nothrow) p2m_weights();
        if (!w) {
            set_error("host allocation failed");
            return P2M_ENOMEM;
        }
        w->device = dev;
        fresh = true;
    } else if (w->device != dev) {
        set_error("handle belongs to device %d, current device is %d", w->device, dev);
        return P2M_EINVAL;
    }
    const int S = static_cast<int>(sets.size());
    const int64_t N = tot.N, n_nodes = tot.n_nodes, nbins = tot.nbins;
    const int64_t nhist = static_cast<int64_t>(nsb) * nch;
    const int64_t ntiles = scan_tile_count(nhist + 1) + 1;
    const bool want32 = (flags & P2M_WEIGHTS_F32) != 0;
    const bool new_table = !w->dsets || w->capSets < S;
    if (!rc) rc = grow(&w->bins.key, N, w->capN);
    if (!rc) rc = grow(&w->bins.rank, N, w->capN);
    if (!rc) rc = grow(&w->bins.perm, N, w->capN);
    if (!rc) rc = grow(&w->bins.pos_s, 2 * N, 2 * w->capN);
    if (!rc) rc = grow(&w->bins.part_pos, 2 * N, 2 * w->capN);
    if (!rc) rc = grow(&w->bins.part_key, N, w->capN);
    if (!rc) rc = grow(&w->bins.part_uid, N, w->capN);
    if (!rc) w->capN = std::max(w->capN, N);
    if (!rc) rc = grow(&w->bins.start, nbins + 2, w->capBins + 2);
    if (!rc) w->capBins = std::max(w->capBins, nbins);
    if (!rc) rc = grow(&w->bins.hist, nhist + 1, w->capHist + 1);
    if (!rc) w->capHist = std::max(w->capHist, nhist);
    if (!rc) rc = grow(&w->bins.tsum, ntiles + 1, w->capTiles + 1);
    if (!rc) w->capTiles = std::max(w->capTiles, ntiles);
    const int64_t n_slots = tot.n_tiles * TILE_N;
    if (!rc) rc = grow(&w->meta, n_slots, w->capSlots);
    if (!rc) rc = grow(&w->slow, n_nodes, w->capNodes);
    if (!rc) rc = grow(&w->rd, n_nodes, w->capNodes);
    if (!rc) rc = grow(&w->tdiag, BUILD_TD * tot.n_tiles, BUILD_TD * (w->capSlots / TILE_N));
    if (!rc && !w->ev_fork) {
        hipError_t e = hipEventCreateWithFlags(&w->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_check(e, "hipEventCreateWithFlags");
    }
    if (!rc) rc = grow(&w->idx, n_slots * KMAX, w->capSlots * KMAX);
    if (!rc) rc = grow(&w->w64, n_slots * KMAX, w->capSlots * KMAX);
    if (!rc) rc = grow(&w->mem, n_slots * KMAX, w->capSlots * KMAX);
    if (!rc && want32) rc = grow(&w->w32, n_slots * KMAX, w->capSlots32 * KMAX);
    if (!rc && want32) w->capSlots32 = std::max(w->capSlots32, n_slots);
    // overflow rows: a small store for the rare rows longer than KMAX
    // (the row stride of every overflow array is capOvf, so they all keep
    // at least that many rows)
    const int64_t novf = std::max({w->capOvf, int64_t{64}, n_nodes / 64});
    const int64_t ovw = KROW - KMAX;
    if (!rc) rc = grow(&w->orow, n_slots, w->capSlots);
    if (!rc) rc = grow(&w->oidx, ovw * novf, ovw * w->capOvf);
    if (!rc) rc = grow(&w->ow64, ovw * novf, ovw * w->capOvf);
    if (!rc) rc = grow(&w->omem, ovw * novf, ovw * w->capOvf);
    if (!rc && want32) rc = grow(&w->ow32, ovw * novf, ovw * w->capOvf32);
    if (!rc) w->capOvf = novf;
    if (!rc && want32) w->capOvf32 = novf;
    if (!rc && (flags & P2M_DETERMINISTIC)) {
        // entry indices are int32 (checked), one per ELL or overflow entry
        const int64_t n_ent = KMAX * n_slots + (KROW - KMAX) * novf;
        if (n_ent >= (int64_t(1) << 31) || N >= (int64_t(1) << 31) - 1) {
            set_error("P2M_DETERMINISTIC: %lld entries / %lld particles exceed the int32 index",
                      static_cast<long long>(n_ent), static_cast<long long>(N));
            rc = P2M_EINVAL;
        }
        const int64_t ntt = transpose_scan_tiles(N) + 1;
        if (!rc) rc = grow(&w->tcnt, N, w->capTN);
        if (!rc) rc = grow(&w->tptr, N + 1, w->capTN + 1);
        if (!rc) w->capTN = std::max(w->capTN, N);
        if (!rc) rc = grow(&w->tent, n_ent, w->capTE);
        if (!rc) rc = grow(&w->tnode, n_ent, w->capTE);
        if (!rc) rc = grow(&w->gent, n_ent, w->capTE);
        if (!rc) w->capTE = std::max(w->capTE, n_ent);
        if (!rc) rc = grow(&w->ttile, ntt, w->capTT);
        if (!rc) w->capTT = std::max(w->capTT, ntt);
    }
    if (!rc && !w->diag) rc = grow(&w->diag, D_COUNT, 0);
    if (!rc) rc = grow(&w->dsets, S, w->capSets);
    if (rc) {
        if (fresh) {
            release(w);
            delete w;
        }
        return rc;
    }
    w->capNodes = std::max(w->capNodes, n_nodes);
    w->capSlots = std::max(w->capSlots, n_slots);
    w->capSets = std::max<int64_t>(w->capSets, S);
    if (new_table || w->hsets.size() != sets.size() ||
        std::memcmp(w->hsets.data(), sets.data(), sizeof(SetDesc) * sets.size()) != 0) {
        // stream-ordered, so kernels still running on the old table finish first
        P2M_HIP(hipMemcpyAsync(w->dsets, sets.data(), sizeof(SetDesc) * S, hipMemcpyHostToDevice, st));
        w->hsets = sets;
    }
    w->S = S;
    w->N = N;
    w->n_nodes = n_nodes;
    w->n_tiles = tot.n_tiles;
    w->flags = flags;
    *wout = w;

    SideWork side{nullptr, w->ev_fork, w->ev_join};
    rc = side_stream(dev, &side.stream);
    if (rc) return rc;
    return launch_build(w, tot, pos, flags, side, st, fp);
}

// Per-device workspace of the fused (recompute) entry points: a weights
// handle and an ELL-shaped gradient buffer, grown on demand and kept for the
// life of the process.  Calls on one device are serialised by a lock.
// An event recorded on the caller's stream after each call makes the next
// call, on whatever stream, wait for the kernels still reading the
// workspace before it is rebuilt.
struct FusedWork {
    std::mutex mu;
    p2m_weights* w = nullptr;
    double* grad_w = nullptr;
    int64_t cap_gw = 0;
    hipEvent_t done = nullptr;
};
// Before reusing the workspace: wait on stream for the previous call's work.
// Under stream capture the graph orders its own nodes (and its replays run
// in stream order), so the event is neither waited for nor recorded there.
bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}
int fused_enter(FusedWork& fw, hipStream_t st) {
    if (capturing(st)) return P2M_OK;
    if (!fw.done) {
        P2M_HIP(hipEventCreateWithFlags(&fw.done, hipEventDisableTiming));
        return P2M_OK;
    }
    P2M_HIP(hipStreamWaitEvent(st, fw.done, 0));
    return P2M_OK;
}
int fused_leave(FusedWork& fw, hipStream_t st, int rc) {
    if (fw.done && !capturing(st)) {
        const hipError_t e = hipEventRecord(fw.done, st);
        if (e != hipSuccess && rc == P2M_OK) return hip_check(e, "hipEventRecord");
    }
    return rc;
}

// Set table of a static-workspace build, stored by a kernel from its argument
// (no host buffer has to outlive the call).
__global__ void k_store_set(SetDesc* d, SetDesc s) { *d = s; }

struct NoAllocWork {
    std::mutex mu;
    unsigned char* base[64] = {};  // device address of `scratch` on each device
    p2m_weights w[64];             // handles whose buffers point into it
};
NoAllocWork& noalloc_work() {
    static NoAllocWork nw;
    return nw;
}
FusedWork& fused_work(int device) {
    static FusedWork works[64];
    return works[device & 63];
}

int check_batch(const p2m_batch* b) {
    if (!b) {
        set_error("batch handle is NULL");
        return P2M_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device) {
        set_error("batch handle belongs to device %d, current device is %d", b->device, dev);
        return P2M_EINVAL;
    }
    return P2M_OK;
}

}  // namespace

extern "C" {


const char* p2m_last_error(void) { return g_err.c_str(); }

const char* p2m_version(void) { return "libp2m 0.1 (gfx950)"; }

int p2m_set_option(const char* name, double value) {
    if (!name) {
        set_error("option name is NULL");
        return P2M_EINVAL;
    }
    if (!std::strcmp(name, "bin_scale") && value >= 0.25 && value <= 8.0) {
        g_tune.bin_scale = value;
    } else if (!std::strcmp(name, "region_h") && value >= 1.0 && value <= 64.0) {
        g_tune.region_h = value;
    } else if (!std::strcmp(name, "fast_radius") && value >= 1.5 && value <= 8.0) {
        g_tune.fast_radius = value;
    } else if (!std::strcmp(name, "closure_radius") && value >= 1.5 && value <= 8.0) {
        g_tune.closure_radius = value;
    } else if (!std::strcmp(name, "levels") && value >= 0.0 && value <= 8.0) {
        g_tune.levels = static_cast<int>(value);
    } else if (!std::strcmp(name, "svd_cond") && value >= 1.0 && value <= 1e16) {
        g_tune.svd_cond = value;
    } else if (!std::strcmp(name, "m2p_ppt") && (value == 1.0 || value == 2.0 || value == 4.0)) {
        g_tune.m2p_ppt = static_cast<int>(value);
    } else {
        set_error("unknown option or value out of range: %s=%g", name, value);
        return P2M_EINVAL;
    }
    return P2M_OK;
}

int p2m_get_option(const char* name, double* value) {
    if (!name || !value) {
        set_error("p2m_get_option: NULL name or value pointer");
        return P2M_EINVAL;
    }
    if (!std::strcmp(name, "bin_scale")) {
        *value = g_tune.bin_scale;
    } else if (!std::strcmp(name, "region_h")) {
        *value = g_tune.region_h;
    } else if (!std::strcmp(name, "fast_radius")) {
        *value = g_tune.fast_radius;
    } else if (!std::strcmp(name, "closure_radius")) {
        *value = g_tune.closure_radius;
    } else if (!std::strcmp(name, "levels")) {
        *value = g_tune.levels;
    } else if (!std::strcmp(name, "svd_cond")) {
        *value = g_tune.svd_cond;
    } else if (!std::strcmp(name, "m2p_ppt")) {
        *value = g_tune.m2p_ppt;
    } else if (!std::strcmp(name, "fast_slots")) {
        *value = fast_slots();
    } else {
        set_error("unknown option: %s", name);
        return P2M_EINVAL;
    }
    return P2M_OK;
}

int build_single(const p2m_mesh* mesh, double h, const double* pos, int64_t N, int flags, p2m_weights** wout,
                 hipStream_t st, const FusedProj* fp) {
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (N < 3 || N >= (int64_t(1) << 28)) {
        set_error("N=%lld out of range [3, 2^28)", static_cast<long long>(N));
        return P2M_EINVAL;
    }
    const int64_t off[2] = {0, N};
    std::vector<SetDesc> sets;
    SetTotals tot;
    rc = make_sets(mesh, &h, off, 1, sets, tot);
    if (rc) return rc;
    return build_sets(sets, tot, pos, flags, wout, st, fp);
}

int p2m_build_weights(const p2m_mesh* mesh, double h, const double* pos, int64_t N, int flags,
                      p2m_weights** wout, void* stream) {
    return build_single(mesh, h, pos, N, flags, wout, static_cast<hipStream_t>(stream), nullptr);
}

int p2m_batch_create(const p2m_mesh* meshes, const double* h, int S, const int64_t* set_offsets, p2m_batch** out) {
    if (!out) {
        set_error("output handle pointer is NULL");
        return P2M_EINVAL;
    }
    *out = nullptr;
    if (!meshes || !h || !set_offsets) {
        set_error("meshes / h / set_offsets is NULL");
        return P2M_EINVAL;
    }
    if (S < 1 || S > P2M_MAX_SETS) {
        set_error("S=%d out of range [1, %d]", S, P2M_MAX_SETS);
        return P2M_EINVAL;
    }
    p2m_batch* b = new (std::nothrow) p2m_batch();
    if (!b) {
        set_error("host allocation failed");
        return P2M_ENOMEM;
    }
    int rc = make_sets(meshes, h, set_offsets, S, b->sets, b->tot);
    if (!rc) {
        b->meshes.assign(meshes, meshes + S);
        b->h.assign(h, h + S);
        b->off.assign(set_offsets, set_offsets + S + 1);
        hipError_t e = hipGetDevice(&b->device);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&b->dsets), sizeof(SetDesc) * S);
        if (e == hipSuccess)
            e = hipMemcpy(b->dsets, b->sets.data(), sizeof(SetDesc) * S, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_check(e, "p2m_batch_create");
    }
    if (rc) {
        if (b->dsets) (void)hipFree(b->dsets);
        delete b;
        return rc;
    }
    *out = b;
    return P2M_OK;
}

int p2m_batch_shape(const p2m_batch* b, int64_t* n_nodes, int64_t* n_particles, int64_t* node_offsets) {
    if (!b) {
        set_error("batch handle is NULL");
        return P2M_EINVAL;
    }
    if (n_nodes) *n_nodes = b->tot.n_nodes;
    if (n_particles) *n_particles = b->tot.N;
    if (node_offsets) {
        for (int s = 0; s < b->S(); ++s) node_offsets[s] = b->sets[s].n0;
        node_offsets[b->S()] = b->tot.n_nodes;
    }
    return P2M_OK;
}

void p2m_batch_destroy(p2m_batch* b) {
    if (!b) return;
    if (b->dsets) (void)hipFree(b->dsets);
    delete b;
}

int p2m_build_weights_batched(const p2m_batch* b, const double* pos, int flags, p2m_weights** wout, void* stream) {
    int rc = check_batch(b);
    if (rc) return rc;
    std::vector<SetDesc> sets;
    SetTotals tot;
    // recomputed so that the current tuning options apply
    rc = make_sets(b->meshes.data(), b->h.data(), b->off.data(), b->S(), sets, tot);
    if (rc) return rc;
    return build_sets(sets, tot, pos, flags, wout, static_cast<hipStream_t>(stream));
}

int p2m_weights_diag(const p2m_weights* w, p2m_diag* d, void* stream) {
    int rc = check_handle(w);
    if (rc) return rc;
    if (!d) {
        set_error("diag is NULL");
        return P2M_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long h[D_COUNT];
    P2M_HIP(hipMemcpyAsync(h, w->diag, sizeof h, hipMemcpyDeviceToHost, st));
    P2M_HIP(hipStreamSynchronize(st));
    d->interior_nodes = static_cast<int64_t>(h[D_INTERIOR]);
    d->closure_nodes = static_cast<int64_t>(h[D_CLOSURE]);
    d->outside_hull_nodes = static_cast<int64_t>(h[D_OUTSIDE]);
    d->rank_deficient = static_cast<int64_t>(h[D_RANKDEF]);
    d->cap_overflow = static_cast<int64_t>(h[D_CAP]);
    d->escalated_nodes = static_cast<int64_t>(h[D_ESCALATED]);
    d->global_nodes = static_cast<int64_t>(h[D_GLOBAL]);
    d->near_degenerate = static_cast<int64_t>(h[D_NEARDEG]);
    d->bad_particles = static_cast<int64_t>(h[D_BAD]);
    d->failed_nodes = static_cast<int64_t>(h[D_FAILED]);
    d->support_max = static_cast<int32_t>(h[D_SUPMAX]);
    d->duplicate_pairs = static_cast<int64_t>(h[D_DUP]);
    d->slow_nodes = static_cast<int64_t>(h[D_SLOWCNT]);
    d->svd_systems = static_cast<int64_t>(h[D_SVD]);
    {
        const unsigned long long b = h[D_GRAMCOND];
        double g = 0.0;
        std::memcpy(&g, &b, sizeof g);
        d->max_gram_cond = g;
    }
    d->bwd_rank_deficient = static_cast<int64_t>(h[D_BWDSKIP]);
    d->long_rows = static_cast<int64_t>(h[D_OVF]);
    int status = P2M_OK;
    if (d->bad_particles) {
        status = P2M_EDOMAIN;
        set_error("%lld particle(s) outside the mesh or non-finite", static_cast<long long>(d->bad_particles));
    } else if (d->duplicate_pairs) {
        status = P2M_EGEOM;
        set_error("%lld pair(s) of coincident particles", static_cast<long long>(d->duplicate_pairs));
    } else if (d->cap_overflow) {
        status = P2M_ECAP;
        set_error("%lld node(s) exceeded the support cap %d or found the overflow store full",
                  static_cast<long long>(d->cap_overflow), KROW);
    } else if ((w->flags & P2M_STRICT) && d->rank_deficient) {
        status = P2M_EGEOM;
        set_error("%lld rank-deficient moment system(s)", static_cast<long long>(d->rank_deficient));
    } else if (d->failed_nodes) {
        status = P2M_EGEOM;
        set_error("%lld node(s) without weights (degenerate geometry)", static_cast<long long>(d->failed_nodes));
    }
    d->status = status;
    return status;
}

int p2m_weights_export(const p2m_weights* w, int32_t* idx, double* wts, int32_t* cnt, int32_t* tri, void* stream) {
    int rc = check_rows(w);
    if (rc) return rc;
    return export_weights(view(w), idx, wts, cnt, tri, static_cast<hipStream_t>(stream));
}

int p2m_weights_shape(const p2m_weights* w, int64_t* n_nodes, int64_t* n_particles) {
    if (!w) {
        set_error("weights handle is NULL");
        return P2M_EINVAL;
    }
    if (n_nodes) *n_nodes = w->n_nodes;
    if (n_particles) *n_particles = w->N;
    return P2M_OK;
}

int p2m_project(const p2m_weights* w, const void* vals, int C, int dtype, void* mesh_vals, void* stream) {
    int rc = check_rows(w);
    if (!rc) rc = check_vals(vals, C, dtype, "vals", false);
    if (!rc) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (rc) return rc;
    return project(view(w), vals, C, dtype, mesh_vals, static_cast<hipStream_t>(stream));
}

int m2p_interpolate(const p2m_mesh* mesh, const void* mesh_vals, int C, int dtype, const double* pos, int64_t N,
                    void* vals, void* stream) {
    int rc = check_mesh(mesh);
    if (!rc) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (!rc) rc = check_vals(vals, C, dtype, "vals", false);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || N < 1 || N >= (int64_t(1) << 31)) {
        set_error("pos is NULL/misaligned or N=%lld out of range", static_cast<long long>(N));
        return P2M_EINVAL;
    }
    const MeshD m = to_meshd(mesh);
    return m2p(m, nullptr, 1, static_cast<int64_t>(m.nx + 1) * (m.ny + 1), mesh_vals, C, dtype, pos, N, vals,
               static_cast<hipStream_t>(stream), g_tune.m2p_ppt);
}

int p2m_advect(const p2m_mesh* mesh, double* pos, int64_t N, double amp, double dt, void* stream) {
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || N < 1 || N >= (int64_t(1) << 31)) {
        set_error("pos is NULL/misaligned or N=%lld out of range", static_cast<long long>(N));
        return P2M_EINVAL;
    }
    if (!std::isfinite(amp) || !std::isfinite(dt)) {
        set_error("amp and dt must be finite");
        return P2M_EINVAL;
    }
    return advect_midpoint(to_meshd(mesh), pos, N, amp, dt, static_cast<hipStream_t>(stream), false);
}

int p2m_advect_periodic(const p2m_mesh* mesh, double* pos, int64_t N, double amp, double dt, void* stream) {
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || N < 1 || N >= (int64_t(1) << 31)) {
        set_error("pos is NULL/misaligned or N=%lld out of range", static_cast<long long>(N));
        return P2M_EINVAL;
    }
    if (!std::isfinite(amp) || !std::isfinite(dt)) {
        set_error("amp and dt must be finite");
        return P2M_EINVAL;
    }
    return advect_midpoint(to_meshd(mesh), pos, N, amp, dt, static_cast<hipStream_t>(stream), true);
}

int m2p_interpolate_batched(const p2m_batch* b, const void* mesh_vals, int C, int dtype, const double* pos,
                            void* vals, void* stream) {
    int rc = check_batch(b);
    if (!rc) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (!rc) rc = check_vals(vals, C, dtype, "vals", false);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16)) {
        set_error("pos is NULL or misaligned");
        return P2M_EINVAL;
    }
    return m2p(MeshD{}, b->dsets, b->S(), b->tot.n_nodes, mesh_vals, C, dtype, pos, b->tot.N, vals,
               static_cast<hipStream_t>(stream), g_tune.m2p_ppt);
}

int m2p_interpolate_backward(const p2m_mesh* mesh, const void* mesh_vals, int C, int dtype, const double* pos,
                             int64_t N, const void* grad_vals, void* grad_mesh, double* grad_pos, void* stream) {
    int rc = check_mesh(mesh);
    if (!rc) rc = check_vals(grad_vals, C, dtype == P2M_BF16 ? P2M_F32 : dtype, "grad_vals", true);
    if (!rc && grad_mesh) rc = check_vals(grad_mesh, C, dtype, "grad_mesh", true);
    if (!rc && grad_pos) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || N < 1 || N >= (int64_t(1) << 31)) {
        set_error("pos is NULL/misaligned or N=%lld out of range", static_cast<long long>(N));
        return P2M_EINVAL;
    }
    if (grad_pos && !aligned(grad_pos, 16)) {
        set_error("grad_pos is misaligned");
        return P2M_EINVAL;
    }
    const MeshD m = to_meshd(mesh);
    return m2p_backward(m, nullptr, 1, static_cast<int64_t>(m.nx + 1) * (m.ny + 1), mesh_vals, C, dtype, pos, N,
                        grad_vals, grad_mesh, grad_pos, static_cast<hipStream_t>(stream));
}

int m2p_interpolate_backward_batched(const p2m_batch* b, const void* mesh_vals, int C, int dtype,
                                     const double* pos, const void* grad_vals, void* grad_mesh, double* grad_pos,
                                     void* stream) {
    int rc = check_batch(b);
    if (!rc) rc = check_vals(grad_vals, C, dtype == P2M_BF16 ? P2M_F32 : dtype, "grad_vals", true);
    if (!rc && grad_mesh) rc = check_vals(grad_mesh, C, dtype, "grad_mesh", true);
    if (!rc && grad_pos) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || (grad_pos && !aligned(grad_pos, 16))) {
        set_error("pos / grad_pos NULL or misaligned");
        return P2M_EINVAL;
    }
    return m2p_backward(MeshD{}, b->dsets, b->S(), b->tot.n_nodes, mesh_vals, C, dtype, pos, b->tot.N, grad_vals,
                        grad_mesh, grad_pos, static_cast<hipStream_t>(stream));
}

int m2p_interpolate_backward_binned(const p2m_weights* w, const void* mesh_vals, int C, int dtype,
                                    const double* pos, const void* grad_vals, void* grad_mesh, double* grad_pos,
                                    void* stream) {
    int rc = check_handle(w);
    if (!rc) rc = check_vals(grad_vals, C, dtype == P2M_BF16 ? P2M_F32 : dtype, "grad_vals", true);
    if (!rc && grad_mesh) rc = check_vals(grad_mesh, C, dtype, "grad_mesh", true);
    if (!rc && grad_pos) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || (grad_pos && !aligned(grad_pos, 16))) {
        set_error("pos / grad_pos NULL or misaligned");
        return P2M_EINVAL;
    }
    return m2p_backward_binned(view(w), mesh_vals, C, dtype, pos, grad_vals, grad_mesh, grad_pos,
                               static_cast<hipStream_t>(stream));
}

int p2m_project_backward(const p2m_weights* w, const void* grad_mesh, int C, int dtype, const void* vals,
                         void* grad_vals, double* grad_w, void* stream) {
    int rc = check_rows(w);
    if (!rc) rc = check_vals(grad_mesh, C, dtype, "grad_mesh", true);
    if (!rc && grad_vals) rc = check_vals(grad_vals, C, dtype == P2M_BF16 ? P2M_F32 : dtype, "grad_vals", false);
    if (!rc && grad_w) rc = check_vals(vals, C, dtype, "vals", false);
    if (rc) return rc;
    if (grad_w && !aligned(grad_w, 8)) {
        set_error("grad_w is misaligned");
        return P2M_EINVAL;
    }
    return project_backward(view(w), grad_mesh, C, dtype, vals, grad_vals, grad_w, static_cast<hipStream_t>(stream));
}

int p2m_build_weights_backward(const p2m_weights* w, const double* pos, const double* grad_w, double* grad_pos,
                               void* stream) {
    int rc = check_rows(w);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || !grad_w || !aligned(grad_w, 8) || !grad_pos || !aligned(grad_pos, 16)) {
        set_error("pos / grad_w / grad_pos NULL or misaligned");
        return P2M_EINVAL;
    }
    if (w->flags & P2M_LINEAR) {
        set_error("weights built with P2M_LINEAR: position gradients are not provided");
        return P2M_EINVAL;
    }
    return build_backward(view(w), pos, grad_w, grad_pos, static_cast<hipStream_t>(stream),
                          (w->flags & P2M_PERIODIC) != 0);
}

const p2m_weights* p2m_fused_handle(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    return fused_work(dev).w;
}

int p2m_project_fused(const p2m_mesh* mesh, double h, const double* pos, int64_t N, const void* vals, int C,
                      int dtype, void* mesh_vals, void* stream) {
    int rc = check_vals(vals, C, dtype, "vals", false);
    if (!rc) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (rc) return rc;
    int dev = 0;
    P2M_HIP(hipGetDevice(&dev));
    FusedWork& fw = fused_work(dev);
    std::lock_guard<std::mutex> lock(fw.mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = fused_enter(fw, st);
    if (rc) return rc;
    const int flags = dtype == P2M_F64 ? 0 : P2M_WEIGHTS_F32;
    if (C <= FUSED_CMAX) {
        // the rows of the fast path are projected as they are weighted; the
        // rest (exact and rank-revealing paths) from their stored weights
        const FusedProj fp{vals, C, dtype, mesh_vals};
        rc = build_single(mesh, h, pos, N, flags, &fw.w, st, &fp);
        if (!rc) rc = project_listed(view(fw.w), fw.w->slow, vals, C, dtype, mesh_vals, st);
    } else {
        rc = build_single(mesh, h, pos, N, flags, &fw.w, st, nullptr);
        if (!rc) rc = p2m_project(fw.w, vals, C, dtype, mesh_vals, stream);
    }
    return fused_leave(fw, st, rc);
}

int p2m_backward_fused(const p2m_mesh* mesh, double h, const double* pos, int64_t N, const void* vals, int C,
                       int dtype, const void* grad_mesh, void* grad_vals, double* grad_pos, void* stream) {
    int rc = check_vals(grad_mesh, C, dtype, "grad_mesh", true);
    if (!rc && grad_pos) rc = check_vals(vals, C, dtype, "vals", false);
    if (rc) return rc;
    if (grad_pos && !aligned(grad_pos, 16)) {
        set_error("grad_pos is misaligned");
        return P2M_EINVAL;
    }
    int dev = 0;
    P2M_HIP(hipGetDevice(&dev));
    FusedWork& fw = fused_work(dev);
    std::lock_guard<std::mutex> lock(fw.mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = fused_enter(fw, st);
    if (rc) return rc;
    rc = p2m_build_weights(mesh, h, pos, N, dtype == P2M_F64 ? 0 : P2M_WEIGHTS_F32, &fw.w, stream);
    double* gw = nullptr;
    if (!rc && grad_pos) {
        const int64_t need = fw.w->n_nodes * KROW;
        rc = grow(&fw.grad_w, need, fw.cap_gw);
        if (!rc) {
            fw.cap_gw = std::max(fw.cap_gw, need);
            gw = fw.grad_w;
        }
    }
    if (!rc && (grad_vals || gw)) rc = p2m_project_backward(fw.w, grad_mesh, C, dtype, vals, grad_vals, gw, stream);
    if (!rc && gw) rc = p2m_build_weights_backward(fw.w, pos, gw, grad_pos, stream);
    return fused_leave(fw, st, rc);
}

int p2m_project_fused_noalloc(const p2m_mesh* mesh, double h, const double* pos, int64_t N, const void* vals,
                              int C, int dtype, void* mesh_vals, void* stream) {
    int rc = check_mesh(mesh);
    if (!rc) rc = check_vals(vals, C, dtype, "vals", false);
    if (!rc) rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (rc) return rc;
    if (N < 3 || N > NA_MAX_N) {
        set_error("p2m_project_fused_noalloc: N=%lld outside [3, %lld] (the static workspace's limit)",
                  static_cast<long long>(N), static_cast<long long>(NA_MAX_N));
        return P2M_EINVAL;
    }
    const int64_t off[2] = {0, N};
    std::vector<SetDesc> sets;
    SetTotals tot;
    rc = make_sets(mesh, &h, off, 1, sets, tot);
    const int flags = dtype == P2M_F64 ? 0 : P2M_WEIGHTS_F32;
    if (!rc) rc = check_build(sets, pos, flags);
    if (rc) return rc;
    int nch = 0, sbs = 0, nsb = 0;
    rc = bin_layout(tot.N, tot.nbins, &nch, &sbs, &nsb);
    if (rc) return rc;
    const int64_t nhist = static_cast<int64_t>(nsb) * nch;
    if (tot.n_tiles > NA_MAX_TILES || tot.nbins > NA_MAX_BINS || nhist > NA_MAX_HIST ||
        scan_tile_count(nhist + 1) + 1 > NA_MAX_TSUM) {
        set_error("p2m_project_fused_noalloc: mesh of %lld node tiles or %lld bins (h=%g) exceeds the static "
                  "workspace (at most %lld tiles of 8 x 8 nodes and %lld bins)",
                  static_cast<long long>(tot.n_tiles), static_cast<long long>(tot.nbins), h,
                  static_cast<long long>(NA_MAX_TILES), static_cast<long long>(NA_MAX_BINS));
        return P2M_EINVAL;
    }
    int dev = 0;
    P2M_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device %d out of range", dev);
        return P2M_EINVAL;
    }
    NoAllocWork& nw = noalloc_work();
    std::lock_guard<std::mutex> lock(nw.mu);
    p2m_weights* w = &nw.w[dev];
    if (!nw.base[dev]) {
        // this device's copy of the array: its device address, taken once
        void* ptr = nullptr;
        P2M_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        unsigned char* b = static_cast<unsigned char*>(ptr);
        w->device = dev;
        w->bins.key = reinterpret_cast<uint32_t*>(b + NA.key);
        w->bins.rank = reinterpret_cast<int32_t*>(b + NA.rank);
        w->bins.perm = reinterpret_cast<int32_t*>(b + NA.perm);
        w->bins.pos_s = reinterpret_cast<double*>(b + NA.pos_s);
        w->bins.part_pos = reinterpret_cast<double*>(b + NA.part_pos);
        w->bins.part_key = reinterpret_cast<uint32_t*>(b + NA.part_key);
        w->bins.part_uid = reinterpret_cast<int32_t*>(b + NA.part_uid);
        w->bins.start = reinterpret_cast<int32_t*>(b + NA.start);
        w->bins.hist = reinterpret_cast<int32_t*>(b + NA.hist);
        w->bins.tsum = reinterpret_cast<int32_t*>(b + NA.tsum);
        w->meta = reinterpret_cast<uint32_t*>(b + NA.meta);
        w->slow = reinterpret_cast<int32_t*>(b + NA.slow);
        w->rd = reinterpret_cast<int32_t*>(b + NA.rd);
        w->tdiag = reinterpret_cast<int32_t*>(b + NA.tdiag);
        w->idx = reinterpret_cast<int32_t*>(b + NA.idx);
        w->w64 = reinterpret_cast<double*>(b + NA.w64);
        w->w32 = reinterpret_cast<float*>(b + NA.w32);
        w->mem = b + NA.mem;
        w->orow = reinterpret_cast<int32_t*>(b + NA.orow);
        w->oidx = reinterpret_cast<int32_t*>(b + NA.oidx);
        w->ow64 = reinterpret_cast<double*>(b + NA.ow64);
        w->ow32 = reinterpret_cast<float*>(b + NA.ow32);
        w->omem = b + NA.omem;
        w->capOvf = w->capOvf32 = NA_OVF;
        w->diag = reinterpret_cast<unsigned long long*>(b + NA.diag);
        w->dsets = reinterpret_cast<SetDesc*>(b + NA.sets);
        nw.base[dev] = b;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    w->S = 1;
    w->N = tot.N;
    w->n_nodes = tot.n_nodes;
    w->n_tiles = tot.n_tiles;
    w->flags = flags;
    k_store_set<<<1, 1, 0, st>>>(w->dsets, sets[0]);
    P2M_HIP(hipGetLastError());
    // no side stream: the exact path runs on the caller's stream
    const SideWork side{nullptr, nullptr, nullptr};
    rc = launch_build(w, tot, pos, flags, side, st);
    if (!rc) rc = p2m_project(w, vals, C, dtype, mesh_vals, stream);
    return rc;
}

int p2m_mesh_qcsf_create(const p2m_mesh* mesh, p2m_mesh_qcsf** out, void* stream) {
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (!out) {
        set_error("out is NULL");
        return P2M_EINVAL;
    }
    *out = nullptr;
    auto* q = new (std::nothrow) p2m_mesh_qcsf();
    if (!q) {
        set_error("out of host memory");
        return P2M_ENOMEM;
    }
    q->m = to_meshd(mesh);
    q->E = mesh_edge_count(q->m);
    rc = grow(&q->idx, q->E * MESH_SUP, 0);
    if (!rc) rc = grow(&q->coef, q->E * MESH_SUP, 0);
    if (!rc) rc = mesh_edge_table(q->m, q->idx, q->coef, static_cast<hipStream_t>(stream));
    if (rc) {
        p2m_mesh_qcsf_destroy(q);
        return rc;
    }
    *out = q;
    return P2M_OK;
}

int p2m_mesh_qcsf_create_periodic(const p2m_mesh* mesh, p2m_mesh_qcsf** out, void* stream) {
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (mesh->nx < 4 || mesh->ny < 4) {
        set_error("a periodic box needs at least 4 cells per side (nx=%d ny=%d)", mesh->nx, mesh->ny);
        return P2M_EINVAL;
    }
    rc = p2m_mesh_qcsf_create(mesh, out, stream);
    if (!rc) (*out)->per = true;
    return rc;
}

int m2p_interpolate_qcsf(const p2m_mesh_qcsf* q, const void* mesh_vals, int C, int dtype, const double* pos,
                         int64_t N, void* vals, void* stream) {
    if (!q || !q->idx || !q->coef) {
        set_error("invalid mesh-function handle");
        return P2M_EINVAL;
    }
    int rc = check_vals(mesh_vals, C, dtype, "mesh_vals", true);
    if (!rc) rc = check_vals(vals, C, dtype, "vals", false);
    if (rc) return rc;
    if (!pos || !aligned(pos, 16) || N < 1 || N >= (int64_t(1) << 31)) {
        set_error("pos is NULL/misaligned or N=%lld out of range", static_cast<long long>(N));
        return P2M_EINVAL;
    }
    return m2p_qcsf(q->m, q->idx, q->coef, mesh_vals, C, dtype, pos, N, vals, static_cast<hipStream_t>(stream),
                    q->per);
}

void p2m_mesh_qcsf_destroy(p2m_mesh_qcsf* q) {
    if (!q) return;
    if (q->idx) (void)hipFree(q->idx);
    if (q->coef) (void)hipFree(q->coef);
    delete q;
}

void p2m_weights_destroy(p2m_weights* w) {
    if (!w) return;
    release(w);
    delete w;
}

}  // extern "C"
