// Host-side launchers of the HIP kernels (internal to libp2m).
#pragma once

#include "common.h"

namespace p2m {

// ---- optional event timing of kernel groups (profile.hip) ----
enum Phase : int {
    PH_BIN = 0, PH_BUILD, PH_PROJECT, PH_M2P, PH_M2P_BWD, PH_PROJECT_BWD, PH_BUILD_BWD,
    PH_BUILD_FAST, PH_BUILD_SLOW, PH_WEIGHTS, PH_K_WEIGHTS, PH_K_WEIGHTS_RD, PH_COUNT
};
class PhaseTimer {
  public:
    PhaseTimer(int phase, hipStream_t st);
    ~PhaseTimer();
    PhaseTimer(const PhaseTimer&) = delete;
    PhaseTimer& operator=(const PhaseTimer&) = delete;

  private:
    int phase_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// ---- utilities (util.hip) ----
int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
int fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t st);
int fill_bytes_zero(void* p, int64_t nbytes, hipStream_t st);

// ---- binning (binning.hip) ----
struct BinBuffers {
    uint32_t* key;       // [N] bin key per particle (user order)
    int32_t* rank;       // [N] rank of a particle in its bin (scratch)
    int32_t* hist;       // [nsb * nch + 1] (super-bin, chunk) counts, scanned in place
    int32_t* tsum;       // [scan tiles + 1]
    double* part_pos;    // [N][2] positions grouped by super-bin
    uint32_t* part_key;  // [N]
    int32_t* part_uid;   // [N]
    int32_t* start;      // [nbins + 2] first sorted slot of every bin
    double* pos_s;       // [N][2] sorted positions
    int32_t* perm;       // [N] sorted -> user id
};
// Chunks, log2(bins per super-bin) and super-bins of the two-level sort.
int bin_layout(int64_t N, int64_t nbins, int* nch, int* sbs, int* nsb);
int64_t scan_tile_count(int64_t n);
// Bins of set s are b0(s) .. b0(s) + nbx nby - 1; key nbins (all sets)
// collects particles outside their set's mesh or non-finite.
int bin_particles(const BinBuffers& b, const double* pos, int64_t N, const SetDesc* sets, int S, int64_t nbins,
                  unsigned long long* diag, hipStream_t st);

// ---- weight build (build.hip) ----
struct BuildOut {
    uint32_t* meta;  // [n_nodes]
    int32_t* idx;    // [KMAX][n_nodes]
    double* w64;     // [KMAX][n_nodes]
    float* w32;      // [KMAX][n_nodes] or null
    uint8_t* mem;    // [KMAX][n_nodes]
    int32_t* orow;   // [n_slots] overflow row of a long row
    int32_t* oidx;   // [KROW - KMAX][n_ovf] entries KMAX.. of long rows
    double* ow64;
    float* ow32;     // or null
    uint8_t* omem;
    int64_t n_ovf;   // overflow rows available
};
// All sets of a batch in one pass: fast quad path, then the weights of its
// rows on the caller's stream while the slow wave path (and the weights of
// its rows) runs on the side stream; sets[S] is device memory, n_tiles the
// 8 x 8 node tiles of all sets.
// A second stream (per device, owned by the library) and the two events
// that fork it from and join it back to the caller's stream.
struct SideWork {
    hipStream_t stream;
    hipEvent_t fork, join;
};
int side_stream(int device, hipStream_t* out);
// fast_slots: candidate slots per lane of the fast pass (7, 8 or 10); slow, rd:
// row-slot lists (capacity n_nodes); tdiag: per-tile records
// [n_tiles][BUILD_TD]; svd_kappa: condition estimate above which a system
// goes to the rank-revealing solver; linear: interior rows are the
// triangle's barycentric coordinates alone.
constexpr int BUILD_TD = 5;
// Fused build (fp non-null; bounded box only): the weights pass adds each
// row it finishes into mesh value `out` at once and stores no weights for
// it; the rows of the exact and rank-revealing paths keep stored weights and
// are projected afterwards by project_listed.
constexpr int FUSED_CMAX = 4;  // channels of a fused build (more: build, then project)
struct FusedProj {
    const void* vals;
    int C;
    int dtype;
    void* out;
};
int build_weights(const BinBuffers& b, const SetDesc* sets, int S, int64_t n_tiles, int64_t n_nodes,
                  const BuildOut& out, int levels, int fast_slots, int32_t* slow, int32_t* rd, int32_t* tdiag,
                  unsigned long long* diag, const SideWork& side, hipStream_t st, bool linear,
                  bool periodic, double svd_kappa, const FusedProj* fp = nullptr);

// ---- projection and interpolation (project.hip, m2p.hip) ----
int project(const WeightsView& w, const void* vals, int C, int dtype, void* mesh_vals, hipStream_t st);
int project_backward(const WeightsView& w, const void* grad_mesh, int C, int dtype, const void* vals,
                     void* grad_vals, double* grad_w, hipStream_t st);
// After a fused build: the rows on the slow-path list and the rank-revealing
// list, projected from their stored weights.
int project_listed(const WeightsView& w, const int32_t* slow, const void* vals, int C, int dtype, void* mesh_vals,
                   hipStream_t st);
// sets == nullptr: one mesh m; else particles/nodes of set s start at
// sets[s].p0 / sets[s].n0 and m is ignored.  n_nodes: all sets.
// Mesh-side quadratically consistent functions: edge count and the table of
// every mesh edge's support node ids and coefficients [E][MESH_SUP] (build.hip),
// and M2P with them (m2p.hip).
constexpr int MESH_SUP = 10;
int64_t mesh_edge_count(const MeshD& m);
int mesh_edge_table(const MeshD& m, int32_t* idx, double* coef, hipStream_t st);
int m2p_qcsf(const MeshD& m, const int32_t* idx, const double* coef, const void* mesh_vals, int C, int dtype,
             const double* pos, int64_t N, void* vals, hipStream_t st, bool periodic);
// One explicit midpoint step of every particle in the cellular flow of the
// mesh box, clamped into the box (advect.hip).
int advect_midpoint(const MeshD& m, double* pos, int64_t N, double amp, double dt, hipStream_t st,
                    bool periodic);
// m2p_ppt: particles per thread (1, 2 or 4), a performance option.
int m2p(const MeshD& m, const SetDesc* sets, int S, int64_t n_nodes, const void* mesh_vals, int C, int dtype,
        const double* pos, int64_t N, void* vals, hipStream_t st, int m2p_ppt = 1);
// M2P adjoint at the particles of a weights handle (built from `pos`): grad_mesh
// gathered per node through the handle's binning, grad_pos per particle.
int m2p_backward_binned(const WeightsView& wv, const void* mesh_vals, int C, int dtype, const double* pos,
                        const void* grad_vals, void* grad_mesh, double* grad_pos, hipStream_t st);
int m2p_backward(const MeshD& m, const SetDesc* sets, int S, int64_t n_nodes, const void* mesh_vals, int C,
                 int dtype, const double* pos, int64_t N, const void* grad_vals, void* grad_mesh, double* grad_pos,
                 hipStream_t st);

// ---- particle-major index of the entries (transpose.hip) ----
// Scan tiles of the per-particle counts (tsum needs one more entry).
int64_t transpose_scan_tiles(int64_t N);
// cnt [N] scratch, ptr [N + 1], ent and nodes [n_ent], tsum [tiles + 1].
int build_transpose(const WeightsView& w, int32_t* cnt, int32_t* ptr, int32_t* ent, int32_t* nodes, int32_t* tsum,
                    hipStream_t st);
// P2M^t gathered per particle through the index (grad_vals overwritten).
int project_backward_gather(const WeightsView& w, const void* grad_mesh, int C, int dtype, void* grad_vals,
                            hipStream_t st);
// grad_pos[u] += the per-entry position derivatives in w.gent of particle u.
int gather_entry_grads(const WeightsView& w, double* grad_pos, hipStream_t st);

// ---- adjoint of the weights (adjoint.hip) ----
int build_backward(const WeightsView& w, const double* pos, const double* grad_w, double* grad_pos,
                   hipStream_t st, bool periodic);
int export_weights(const WeightsView& w, int32_t* idx, double* wts, int32_t* cnt, int32_t* tri,
                   hipStream_t st);

}  // namespace p2m
