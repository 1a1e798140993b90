// sph_internal.h -- shared definitions of the HIP kernels and the host
// runtime of libsph.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

constexpr int kBlock = 256;   // threads per workgroup of the per-particle kernels
constexpr int kMaxBodies = 16;

// Uniform grid of the neighbour search (Sec. 5.6 prefix-sum grid).
struct Grid {
    float o[3];      // origin fl32(domain_min - cell)
    float inv;       // fl32(1 / cell)
    int32_t n[3];    // cells per axis
    float h2;        // neighbour predicate d^2 < h2
};

// Constants of the cubic spline with support h (Sec. 3.2) and the fluid mass.
struct Kern {
    float h, inv_h;
    float k;         // 8 / (pi h^3): W = k f(q)
    float kg;        // 6 k / h: dW/dr = kg f'(q) / 6 with f' the polynomial slope
    float m;         // fluid particle mass rho0 (2r)^3
    float rho0;
    float alpha_max;  // cap of the DFSPH factor alpha (0: none)
    float d_min;      // alpha = 0 unless its denominator exceeds this (1e-12 of a bulk particle's)
};

// neighbour statistics: [min, max, sum, sum_fluid]
constexpr int kNStats = 4;

// Device-side state of one Jacobi solve (Algorithm 2): the host queues
// iterations ahead and every pass of an iteration that is no longer due
// returns at once, so the stop rule needs no host round trip per iteration.
struct SolveCtl {
    double err;          // error after the last predict pass
    double scale;        // err = scale * (FP64 sum of the clamped deviations)
    double eta;
    int32_t iters;       // iterations done
    int32_t go;          // 1 while another iteration is due
    int32_t forced;      // >= 0: exactly this many iterations
    int32_t max_iters;
    double eta_max;      // > 0: also iterate while err_max > eta_max
    double max_scale;    // err_max = max_scale * (largest clamped deviation)
    double err_max;
};

// Device-side state of the implicit-viscosity CG (Eq. 19): as SolveCtl, the
// host queues iterations and every kernel of an iteration past the stop does
// nothing.  alpha and beta are the FP64 step ratios the next kernels use.
struct CgCtl {
    double rz;           // r.z of the current residual
    double alpha;        // step length of the last iteration
    double beta;         // direction weight of the last iteration
    double rr;           // r.r after the last update
    double bnorm;        // |b|
    double thresh;       // tol |b|: stop when |r| <= thresh
    int32_t iters;
    int32_t go;
    int32_t max_iters;
    int32_t pad;
};

// What the host reads after a stream synchronisation: the finishing kernels
// store it straight into pinned host memory, so no copy is queued for it.
struct HostStatus {
    SolveCtl solve;                        // the control block after the last finish
    CgCtl cg;                              // the CG control block after the last finish
    uint32_t flags;                        // build flags (bit 0 capacity, bit 1 cell > 4096)
    uint32_t vmax_bits;                    // max |v|^2 (FP32 bits) of the CFL pass
    unsigned long long nstats[kNStats];    // neighbour statistics of the last build
    double rigid[6 * kMaxBodies];          // force and torque per body
};

// Pose of one rigid body for the boundary update (FP64).
struct BodyPose {
    double com[3];
    double R[9];
    double vel[3];
    double omega[3];
};

// A body's mass and world inertia during a step of the strong coupling
// (the pose, and so the inertia, stays fixed until the step's end).
struct BodyDyn {
    double mass;
    double Iw[9];
    double Iwinv[9];
};

// ---------------------------------------------------------------- launchers
// Every launcher queues on `s` and returns hipGetLastError().  Reductions
// store one partial per workgroup in `partials` (reduction_blocks(n) entries
// times the outputs) and finish in a one-workgroup kernel.
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);

// counting sort by (cell key, id)
hipError_t launch_keys_hist(const float4* x, int64_t n, Grid g, uint32_t* key, uint32_t* slot,
                            uint32_t* count, hipStream_t s);
hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* partials,
                                 hipStream_t s);   // out[0..n], out[n] = total
hipError_t launch_scatter(const uint32_t* key, const uint32_t* slot, const uint32_t* start, int64_t n,
                          uint32_t* src, hipStream_t s);
hipError_t launch_cell_sort(const uint32_t* start, int64_t ncell, uint32_t* src, const int32_t* id,
                            uint32_t* flags, hipStream_t s);
// dv/dvo (nullable): the implicit-viscosity correction, carried along;
// xo.w = Kv / rho (the next divergence warm start)
hipError_t launch_gather_fluid(const uint32_t* src, int64_t n, const float4* x, const float4* v, const float* K,
                               const float* Kv, const float* rho, const int32_t* id, const float4* dv, float4* xo,
                               float4* vo, float* Ko, float* Kvo, float* rhoo, int32_t* ido, float4* dvo,
                               hipStream_t s);
hipError_t launch_gather_boundary(const uint32_t* src, int64_t n, const float4* x, const float4* v,
                                  const int32_t* id, float4* xo, float4* vo, int32_t* ido, hipStream_t s);

// neighbour lists, neighbour-major [cap][n]
hipError_t launch_nbr_build(const float4* x, int64_t nf, const float4* xb, const uint32_t* start_f,
                            const uint32_t* start_b, Grid g, uint32_t* nlist, uint32_t* ncnt, int32_t capf,
                            uint32_t* blist, uint32_t* bcnt, int32_t capb, uint32_t* flags,
                            unsigned long long* partials, HostStatus* host, hipStream_t s);
hipError_t launch_boundary_psi(float4* xb, int64_t nb, const uint32_t* start_b, Grid g, Kern kc, hipStream_t s);

// the step
hipError_t launch_max_v2(const float4* v, int64_t n, uint32_t* partials, HostStatus* host, hipStream_t s);
// density, alpha; with warm_factor > 0 also the divergence warm start's
// pressure from x.w (Kv_prev / rho_prev) and Kv = warm_factor x.w rho
// din (nullable): also the density change rate of the input velocity v
// (boundary velocities vb, nullable = at rest); then vout must differ from v.
hipError_t launch_density_alpha(int64_t nf, float4* x, const float4* v, float4* vout, const uint32_t* nlist,
                                const uint32_t* ncnt, const float4* xb, const float4* vb, const uint32_t* blist,
                                const uint32_t* bcnt, Kern kc, float* rho, float* alpha, float4* v_in, float* Kv,
                                float dt, float warm_factor, float pci_c, float* din, hipStream_t s);
// go (nullable): the pass does nothing when *go == 0 (an iteration the
// solve no longer needs).
hipError_t launch_pressure_update(int64_t nf, const float4* x, float4* v, const float* kappa, float* Kacc,
                                  float* kappa_last, const uint32_t* nlist, const uint32_t* ncnt, const float4* xb,
                                  const uint32_t* blist, const uint32_t* bcnt, Kern kc, float dt,
                                  const int32_t* go, hipStream_t s);
// mode 0: divergence (kappa = max(d,0) alpha / dt); mode 1: density
// (kappa = max(rho - rho0 + dt d, 0) alpha / dt^2).  Writes kappa, kappa/rho
// into x.w, and the FP64 sum of the clamped error into *err_out.
// first: the solve's initial predict (always runs); otherwise the pass and
// its finish do nothing once ctl->go == 0.  The finish updates ctl.  dout
// (nullable, mode 0 only): the unclamped divergence d of every particle.
// vb null: every boundary particle is at rest.
hipError_t launch_predict(int mode, int64_t nf, float4* x, const float4* v, const float* rho, const float* alpha,
                          float* kappa, const uint32_t* nlist, const uint32_t* ncnt,
                          const float4* xb, const float4* vb, const uint32_t* blist, const uint32_t* bcnt,
                          Kern kc, float dt, double* partials, SolveCtl* ctl, bool first, float* dout,
                          int* nparts, hipStream_t s);   // the pass only; nparts partials for the finish
// WCSPH equation of state: kappa = max(k ((rho/rho0)^gamma - 1), 0) / rho,
// x.w = kappa/rho, K = 0; nparts partials of max(rho - rho0, 0) for a finish
hipError_t launch_eos(int64_t nf, float4* x, const float* rho, float* kappa, float* K, Kern kc, float k, float gamma,
                      double* partials, int* nparts, hipStream_t s);
// One-workgroup finish of a predict pass over nblk partials: the first finish
// of a solve initialises ctl from init; every finish copies ctl to host->solve.
hipError_t launch_solve_finish(const double* partials, int nblk, SolveCtl* ctl, bool first, const SolveCtl& init,
                               HostStatus* host, hipStream_t s);
// non-pressure: v* = v + dt g + viscosity; also sets up the density warm start
// (kappa = warm_factor K, K = 0, x.w = kappa / rho) when setup_warm and not press.
// press: also the pressure pass of the stiffness already in x.w / kappa
// (v* -= dt a_p, K += kappa, kappa_last = kappa when non-null).
// Outputs of the divergence-free solve's first error pass when the
// non-pressure pass takes it over (see k_nonpressure): boundary velocities
// (null: all at rest) and alpha in; kappa_v and kappa_v/rho (kvs, with a
// pressure in the same pass), D rho/Dt (dout, nullable) and the error
// partials out.
struct DivCheck {
    const float4* vb;
    const float* alpha;
    float2* kvs;
    float* dout;
    double* partials;
};

// div (nullable): also take the divergence check; *nparts = its partials.
hipError_t launch_nonpressure(int model, int64_t nf, float4* x, const float4* v, float4* vout, const float* rho,
                              const uint32_t* nlist, const uint32_t* ncnt, Kern kc, float dt, float gx, float gy,
                              float gz, float visc, float* K, float* kappa, float warm_factor, bool setup_warm,
                              bool press, const float4* xb, const uint32_t* blist, const uint32_t* bcnt,
                              float* kappa_last, const DivCheck* div, int* nparts, hipStream_t s);
hipError_t launch_div_resume(int64_t nf, float4* x, float* kappa, float* K, const float2* kvs, const float* Ksaved,
                             hipStream_t s);
// Ksave (nullable): keep a copy of K before it is cleared.
hipError_t launch_warm_setup(int64_t nf, float4* x, const float* rho, float* K, float* kappa, float warm_factor,
                             float* Ksave, hipStream_t s);
// x += dt v; partials (nullable): also max |v|^2 of the new v to host->vmax_bits;
// gate (nullable): both kernels do nothing while *gate != 0
hipError_t launch_integrate(int64_t nf, float4* x, const float4* v, float dt, uint32_t* partials, HostStatus* host,
                            const int32_t* gate, hipStream_t s);
// Strong coupling (one pressure pass): the reaction of the pass on every body
// from each fluid particle's kappa/rho = xw_scale * x.w (Eq. 14), summed into
// ft (force and torque per body) and the step's totals, the bodies'
// velocities advanced by it (FP64, in poses), and their boundary velocities
// refreshed.  Nothing happens when go (nullable) reads 0.
hipError_t launch_rigid_couple(int64_t nf, const float4* x, const uint32_t* blist, const uint32_t* bcnt,
                               float4* xb, float4* vb, const int32_t* bid, const double* local, Kern kc,
                               int32_t nbody, const double* com, int64_t nb, double* partials, float xw_scale,
                               float dt, const int32_t* go, const BodyDyn* dyn, BodyPose* poses, double* ft_total,
                               HostStatus* host, hipStream_t s);
// The bodies' own accelerations in the strong coupling: V += dt g and the
// gyroscopic term w += dt Iw^-1 (-(w x Iw w)), then their boundary velocities.
hipError_t launch_rigid_gravity(int32_t nbody, int64_t nb, float4* xb, float4* vb, const int32_t* bid,
                                const double* local, const BodyDyn* dyn, BodyPose* poses, double gx, double gy,
                                double gz, float dt, hipStream_t s);
hipError_t launch_rigid_force(int64_t nf, const float4* x, const float* rho, const float* K, const float* Kv,
                              const uint32_t* blist, const uint32_t* bcnt, const float4* xb, const float4* vb,
                              Kern kc, int32_t nbody, const double* com, double* partials, HostStatus* host,
                              hipStream_t s);
hipError_t launch_rigid_boundary(int64_t nb, float4* xb, float4* vb, const int32_t* bid, const double* local,
                                 const BodyPose* poses, hipStream_t s);

// implicit viscosity (Eqs. 16-19): M p = p - dt A p and its block-Jacobi
// preconditioner (per particle the upper triangle of the inverse 3x3 block:
// 00, 01, 02, 11, 12, 22 as three float2)
hipError_t launch_visc_precond(int64_t nf, const float4* x, const float* rho, const uint32_t* nlist,
                               const uint32_t* ncnt, Kern kc, float dt, float mu, float2* Pinv, hipStream_t s);
// M p with the volume m/rho taken from p.w; go (nullable): skip when *go == 0;
// partials (nullable): per-workgroup sums of p.(M p), visc_matvec_parts(nf) of them
int visc_matvec_parts(int64_t nf);
hipError_t launch_visc_matvec(int64_t nf, const float4* x, const float4* p, float4* Mp, const uint32_t* nlist,
                              const uint32_t* ncnt, Kern kc, float dt, float mu, const int32_t* go,
                              double* partials, hipStream_t s);
// b = v + dt g, x0 = b + w dvisc (w = m/rho from v.w in both)
hipError_t launch_cg_start(int64_t nf, const float4* v, const float4* dvisc, float4* b, float4* x0, float dt,
                           float gx, float gy, float gz, float w, hipStream_t s);
// dvisc = v* - b
hipError_t launch_visc_correction(int64_t nf, const float4* vs, const float4* b, float4* dvisc, hipStream_t s);
// r = b - M x0, z = P r, p = z, and the control block of iteration 0 in *ctl
// (partials: 3 per workgroup of nf)
hipError_t launch_cg_setup(int64_t nf, const float4* b, const float4* Mx, const float2* Pinv, float4* r, float4* z,
                           float4* p, double* partials, CgCtl* ctl, double tol, int32_t max_iters,
                           HostStatus* host, hipStream_t s);
// The update of one CG iteration after its mat-vec w = M u (with nuw partial
// sums u.w), in the single-reduction form (see k_cg_update): the stop rule
// from the previous update's sums prev_part (not read when first), then
// p, s = M p, x, r, u = P r and the sums r.u, r.r into partials (2 per
// workgroup of nf).  Reads *ctl, writes the next control block *next.
hipError_t launch_cg_iteration(int64_t nf, float4* xv, float4* r, float4* u, float4* p, float4* sv, const float4* w,
                               const float2* Pinv, const CgCtl* ctl, CgCtl* next, const double* prev_part,
                               const double* uw_part, int nuw, double* partials, HostStatus* host, bool first,
                               hipStream_t s);

// learned warm start: the features pass, the learned stiffness, trace targets
// learned-warm-start features from per-particle fields (no neighbour pass):
// (rho - rho0)/rho0, dt d/rho0 (d of the input velocity, from the density pass),
// (n_f + n_b)/26, K_prev dt^2/(alpha rho0), alpha/alpha_ref; feat [nf][5]
hipError_t launch_features(int64_t nf, const float* rho, const float* alpha, const float* K, const uint32_t* ncnt,
                           const uint32_t* bcnt, const float* d, Kern kc, float dt, float alpha_ref, float* feat,
                           hipStream_t s);
hipError_t launch_warm_learned(int64_t nf, float4* x, const float* rho, const float* alpha, const float* y, float* K,
                               float* kappa, float dt, float rho0, hipStream_t s);
hipError_t launch_trace_target(int64_t nf, const float* alpha, const float* K, float dt, float rho0, float* target,
                               hipStream_t s);

// the MLP (sph_mlp.hip)
int mlp_param_count();
int mlp_grad_blocks();
// inference reads operands that launch_mlp_pack prepares from P (mlp_packed_words() words);
// pack again after every change of P
int mlp_packed_words();
hipError_t launch_mlp_pack(const float* P, uint32_t* packed, hipStream_t s);
hipError_t launch_mlp_forward(const uint32_t* packed, const float* feat, int64_t n, float* y, hipStream_t s);
// features, network and start stiffness in one pass (as launch_features,
// launch_mlp_forward and launch_warm_learned in sequence)
hipError_t launch_mlp_warm_start(const uint32_t* packed, int64_t n, float4* x, const float* rho, const float* alpha,
                                 float* K, float* kappa, const uint32_t* ncnt, const uint32_t* bcnt, const float* d,
                                 Kern kc, float dt, float alpha_ref, float* Ksave, hipStream_t s);
hipError_t launch_mlp_grad(const float* P, const float* feat, const float* target, int64_t n, float* part,
                           double* loss_part, float* grad, double* loss_sum, hipStream_t s);
hipError_t launch_mlp_adam(float* P, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t s);

// workgroups of a per-particle launch over n (a multiple of 8)
uint32_t reduction_blocks(int64_t n);

}  // namespace sph
