// Kinematic transport of the particles between projections: the prescribed
// velocity of the paper's kinematic tests, here the cellular flow of
// streamfunction A sin(pi (x - x0)/Lx) sin(pi (y - y0)/Ly) on the mesh box
// (u = dpsi/dy, v = -dpsi/dx: no flow through the walls of a bounded box),
// advanced by one explicit midpoint step and clamped into the box.  In a
// periodic box the flow is A cos(2 pi (x - x0)/Lx) cos(2 pi (y - y0)/Ly)
// (periodic, crossing the box sides) and a moved particle is wrapped back
// into [x0, x0 + Lx) x [y0, y0 + Ly).  One thread per particle, positions
// updated in place.
#include "kernels.h"

namespace p2m {

namespace {

// bounded:  u = ax sin(kx (x - x0)) cos(ky (y - y0)), v = -ay cos(kx (x - x0)) sin(ky (y - y0))
// periodic: u = -ax cos(kx (x - x0)) sin(ky (y - y0)), v = ay sin(kx (x - x0)) cos(ky (y - y0))
struct Flow {
    double x0, y0, x1, y1, kx, ky, ax, ay, lx, ly;
    int per;
};

__device__ __forceinline__ double2 velocity(const Flow& f, double2 p) {
    double sx, cx, sy, cy;
    sincos(f.kx * (p.x - f.x0), &sx, &cx);
    sincos(f.ky * (p.y - f.y0), &sy, &cy);
    if (f.per) return make_double2(-f.ax * cx * sy, f.ay * sx * cy);
    return make_double2(f.ax * sx * cy, -f.ay * cx * sy);
}

// x moved by whole periods into [o, o + L) (one rounding; a result that
// rounds onto the far side is the near one)
__device__ __forceinline__ double wrap1(double x, double o, double L) {
    const double k = floor((x - o) / L);
    const double w = __dadd_rn(x, -__dmul_rn(k, L));
    return w >= __dadd_rn(o, L) ? o : w;
}

__global__ void __launch_bounds__(256) k_advect(Flow f, double dt, double2* __restrict__ pos, int64_t N) {
    const int64_t mu = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (mu >= N) return;
    const double2 p = pos[mu];
    const double2 u0 = velocity(f, p);
    const double2 mid = make_double2(p.x + 0.5 * dt * u0.x, p.y + 0.5 * dt * u0.y);
    const double2 u1 = velocity(f, mid);
    const double x = p.x + dt * u1.x, y = p.y + dt * u1.y;
    if (f.per) pos[mu] = make_double2(wrap1(x, f.x0, f.lx), wrap1(y, f.y0, f.ly));
    else pos[mu] = make_double2(fmin(fmax(x, f.x0), f.x1), fmin(fmax(y, f.y0), f.y1));
}

}  // namespace

int advect_midpoint(const MeshD& m, double* pos, int64_t N, double amp, double dt, hipStream_t st,
                    bool periodic) {
    const double lx = m.nx * m.H, ly = m.ny * m.H;  // the box's sides
    Flow f;
    f.x0 = m.x0;
    f.y0 = m.y0;
    // the box of the binning and of M2P: product, then sum, each rounded
    // (separate statements: no fused multiply-add)
    const double wx = m.nx * m.H, wy = m.ny * m.H;
    f.x1 = m.x0 + wx;
    f.y1 = m.y0 + wy;
    f.lx = lx;
    f.ly = ly;
    f.per = periodic ? 1 : 0;
    const double c = periodic ? 2.0 * M_PI : M_PI;
    f.kx = c / lx;
    f.ky = c / ly;
    f.ax = amp * c / ly;
    f.ay = amp * c / lx;
    const int64_t blocks = (N + 255) / 256;
    k_advect<<<static_cast<unsigned>(blocks), 256, 0, st>>>(f, dt, reinterpret_cast<double2*>(pos), N);
    P2M_HIP(hipGetLastError());
    return P2M_OK;
}

}  // namespace p2m
