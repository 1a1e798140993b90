// sph_api.cpp -- host runtime and C ABI of libsph.so (see include/sph.h).
//
// The context owns the device buffers, drives the kernels of one DFSPH step
// on its stream, runs the convergence loops of the two Jacobi solves
// (Algorithm 2: stop when the FP64-reduced error is at most eta), and
// integrates the rigid bodies on the host in FP64 (weak coupling: their
// velocities are fixed during the fluid solve).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "sph.h"
#include "sph_internal.h"

using sph::BodyPose;
using sph::Grid;
using sph::Kern;

namespace {

thread_local std::string g_create_error;

struct ProfEvent {
    std::string name;
    hipEvent_t a, b;
    double bytes;
};

struct ProfTotal {
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
};

}  // namespace

struct sph_ctx {
    sph_params P{};
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t nf = 0, nb = 0;
    int32_t nr = 0;
    Grid g{};
    Kern kc{};
    float cell = 0.f;
    float pci_c = 0.f;   // PCISPH stiffness factor (0 for the other solvers)
    int64_t ncell = 0;
    int32_t capf = 0, capb = 0;

    // fluid, sorted order
    float4 *x = nullptr, *x2 = nullptr, *v = nullptr, *v2 = nullptr, *v_in = nullptr;
    float *rho = nullptr, *alpha = nullptr, *K = nullptr, *K2 = nullptr, *Kv = nullptr, *Kv2 = nullptr;
    float *kappa = nullptr, *kappa_last = nullptr;
    int32_t *id = nullptr, *id2 = nullptr;
    uint32_t *key = nullptr, *slot = nullptr, *src = nullptr, *count = nullptr, *start_f = nullptr;
    uint32_t *scan_part = nullptr;
    uint32_t *nlist = nullptr, *ncnt = nullptr, *blist = nullptr, *bcnt = nullptr;
    uint32_t *ncnt2 = nullptr, *bcnt2 = nullptr;   // the previous build's counts (read-back after a build ahead)
    // The step's outputs that the sort does not reorder (alpha, kappa_last,
    // v_in, the neighbour counts) stay in the order of the step that wrote
    // them.  out_order says where that order's ids and counts are now: the
    // current id/ncnt/bcnt (no sort since the step), id2/ncnt2/bcnt2 (one
    // sort), or a copy in id_out/ncnt_out/bcnt_out, taken before a second sort
    // overwrites id2.
    enum class OutOrder { Cur, Prev, Saved } out_order = OutOrder::Cur;
    int32_t *id_out = nullptr;
    uint32_t *ncnt_out = nullptr, *bcnt_out = nullptr;
    // boundary, sorted order (xb.w = Psi, vb.w = body id)
    float4 *xb = nullptr, *xb2 = nullptr, *vb = nullptr, *vb2 = nullptr;
    int32_t *bid = nullptr, *bid2 = nullptr;
    uint32_t *bkey = nullptr, *bslot = nullptr, *bsrc = nullptr, *start_b = nullptr;
    double *blocal = nullptr;   // [nb][3] body-frame offsets, original order
    BodyPose *poses = nullptr;
    sph::BodyDyn *dyn = nullptr;   // strong coupling: mass and world inertia per body for the step
    double *ft = nullptr;          // strong coupling: the step's summed reaction, then one pass's [2][6 kMaxBodies]
    bool strong = false;           // strong (interlinked) rigid-fluid coupling
    double *com_dev = nullptr;
    // reductions and flags
    double *red_part = nullptr, *scal = nullptr;
    sph::SolveCtl *ctl = nullptr;                     // device control block of the running solve
    sph::CgCtl *cgc = nullptr;                        // and of the implicit-viscosity CG
    int32_t last_cg = 0;                              // previous step's CG iterations
    int32_t last_iters[2] = {0, 0};                   // previous step's iterations (divergence, density)
    double last_err_max = 0.0;                        // largest predicted compression after the density solve
    int32_t div_calm = 2;                             // steps in a row whose divergence solve did not iterate
    uint32_t *flags = nullptr;
    unsigned long long *nstat_part = nullptr;
    // pinned host memory the finishing kernels write (host view, device address)
    sph::HostStatus *hs = nullptr, *hs_dev = nullptr;
    // implicit viscosity
    float2 *Pinv = nullptr;   // per particle the upper triangle of its inverse diagonal block
    float4 *cg_b = nullptr, *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_Ap = nullptr, *cg_s = nullptr;
    float4 *dvisc = nullptr, *dvisc2 = nullptr;   // previous correction v* - b, sorted order
    float *rho2 = nullptr;                        // density ping-pong
    float2 *div_kvs = nullptr;   // divergence check folded into the non-pressure pass: kappa_v, kappa_v / rho
    float *K_saved = nullptr;    // and K as it was before the warm start's set-up
    double *cg_part = nullptr;                    // CG partial sums (mat-vec, then two update slots)

    std::vector<sph_rigid_desc> rigid;
    std::vector<double> force, torque;
    std::vector<double> local_host;   // [nb][3] body-frame offsets, original order
    std::vector<int32_t> body_host;   // [nb]
    std::vector<std::vector<double>> body_points;   // per body: its particles' body-frame offsets
    std::vector<void *> allocs;
    int64_t dev_bytes = 0;
    // a borrowed arena (sph_scene::device_arena) or, with counting set, no
    // memory at all: dev_alloc only adds up the aligned sizes
    char *arena = nullptr;
    int64_t arena_bytes = 0;
    bool counting = false;

    bool nbr_fresh = false, boundary_dirty = true, sorted_once = false;
    bool vb_moving = false;   // some boundary velocity may be non-zero (rigid bodies, or written)
    // auto_rebuild: the next step's sort and neighbour build were queued at
    // the end of the last step (the per-particle fields the sort does not
    // reorder, and the previous counts, are then read back through id2)
    bool build_ahead = false;
    bool vmax_ready = false;   // hs->vmax_bits holds max |v|^2 of the current v
    unsigned long long nstats[sph::kNStats] = {};   // of the last build
    int64_t step_index = 0;
    float last_dt = 0.f;
    int32_t forced_div = -1, forced_dens = -1;
    double nbr_sum = 0.0, nbr_sum_f = 0.0;
    std::string err;

    // learned warm start and trace capture
    int32_t warm_mode = SPH_WARM_PREVIOUS;
    sph_mlp *mlp = nullptr;
    bool warm_fallback = false;
    float *feat = nullptr, *ybuf = nullptr;
    float *dbuf = nullptr;   // density change rate of the step's input velocity (learned features)
    bool want_d = false;
    float *trace_feat = nullptr, *trace_target = nullptr;
    int64_t trace_cap = 0, trace_rows = 0;

    hipEvent_t build_done = nullptr;   // recorded after a build queued by sph_step
    hipEvent_t vmax_done = nullptr;    // recorded after the CFL reduction at the end of a step

    bool prof = false;
    std::string prof_only;   // empty: every name
    std::vector<ProfEvent> prof_pending;
    std::vector<hipEvent_t> event_pool;
    std::map<std::string, ProfTotal> prof_total;
};

struct sph_mlp {
    hipStream_t stream = nullptr;
    float *P = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *part = nullptr;
    uint32_t *packed = nullptr;   // inference operands prepared from P (after every change of P)
    double *loss_part = nullptr, *loss = nullptr;
    int64_t step = 0;
    bool finite = true;
};

namespace {

int fail(sph_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                           \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail(ctx, SPH_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

template <typename T>
int dev_alloc(sph_ctx *c, T **p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (c->arena || c->counting) {   // 256-byte aligned pieces of the arena
        const int64_t at = c->dev_bytes;
        const int64_t need = ((int64_t)bytes + 255) / 256 * 256;
        if (c->arena && at + need > c->arena_bytes)
            return fail(c, SPH_ERR_OOM, "device arena of " + std::to_string(c->arena_bytes) + " bytes is too small");
        c->dev_bytes += need;
        *p = c->arena ? (T *)(c->arena + at) : nullptr;
        return SPH_OK;
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(c, SPH_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    c->allocs.push_back(q);
    c->dev_bytes += (int64_t)bytes;
    *p = (T *)q;
    return SPH_OK;
}

void free_all(sph_ctx *c) {
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->hs) (void)hipHostFree(c->hs);
    c->hs = nullptr;
    c->hs_dev = nullptr;
    for (auto &e : c->prof_pending) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    c->prof_pending.clear();
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    c->event_pool.clear();
    if (c->build_done) (void)hipEventDestroy(c->build_done);
    if (c->vmax_done) (void)hipEventDestroy(c->vmax_done);
    c->build_done = c->vmax_done = nullptr;
}

hipEvent_t take_event(sph_ctx *c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (an L2 write-back and invalidate
    // around every timed kernel would slow the kernels that follow)
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
}

// ---- profiling -------------------------------------------------------------
struct ProfScope {
    sph_ctx *c;
    ProfEvent ev{};
    bool on;
    ProfScope(sph_ctx *ctx, const char *name, double bytes)
        : c(ctx), on(ctx->prof && (ctx->prof_only.empty() || ctx->prof_only == name)) {
        if (!on) return;
        ev.name = name;
        ev.bytes = bytes;
        ev.a = take_event(c);
        ev.b = take_event(c);
        (void)hipEventRecord(ev.a, c->stream);
    }
    ~ProfScope() {
        if (!on) return;
        (void)hipEventRecord(ev.b, c->stream);
        c->prof_pending.push_back(ev);
    }
};

void prof_resolve(sph_ctx *c) {
    if (c->prof_pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->prof_pending) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e.a, e.b);
        ProfTotal &t = c->prof_total[e.name];
        t.launches += 1;
        t.ms += ms;
        t.bytes += e.bytes;
        c->event_pool.push_back(e.a);
        c->event_pool.push_back(e.b);
    }
    c->prof_pending.clear();
}

// ---- rigid body helpers (FP64) -------------------------------------------
void quat_to_R(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

int upload_poses(sph_ctx *c) {
    if (c->nr == 0) return SPH_OK;
    std::vector<BodyPose> poses(c->nr);
    std::vector<double> com(3 * c->nr);
    for (int b = 0; b < c->nr; ++b) {
        const sph_rigid_desc &s = c->rigid[b];
        quat_to_R(s.quat, poses[b].R);
        for (int a = 0; a < 3; ++a) {
            poses[b].com[a] = s.com[a];
            poses[b].vel[a] = s.vel[a];
            poses[b].omega[a] = s.omega[a];
            com[3 * b + a] = s.com[a];
        }
    }
    HIP_TRY(c, hipMemcpyAsync(c->poses, poses.data(), sizeof(BodyPose) * c->nr, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->com_dev, com.data(), sizeof(double) * 3 * c->nr, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SPH_OK;
}

// Rigid contact in FP64 (the paper takes rigid dynamics from a physics
// engine, Sec. 4.2; this is a frictionless contact model of our own).  The
// bodies' sample points are their contact geometry: a point closer than one
// sampling spacing s = 2r to the interior shrunk by r (the tank), or closer
// than 2s to another body's point, makes a contact with normal n and gap g
// (distance to the plane; point distance minus s).  Each contact asks that
// the point close by at most g within the step, v_n >= -g / dt, with v_n the
// relative normal velocity there.  Projected Gauss-Seidel on accumulated
// normal impulses, 30 sweeps in a fixed order (tank contacts by body, point,
// axis, side; then body pairs a < b by point of a, point of b), applied to
// the velocities the step gave the bodies, at the step's starting pose.
struct Contact {
    int a, b;                 // bodies; b = -1 for the tank
    double n[3], ra[3], rb[3];
    double bias, K, lam;
};

namespace {
double contact_inv_mass(const sph_rigid_desc &s, const double *Iv, const double r[3], const double n[3]) {
    double rn[3];
    cross3(r, n, rn);
    double q = 0.0;
    for (int a = 0; a < 3; ++a) q += rn[a] * (Iv[3 * a] * rn[0] + Iv[3 * a + 1] * rn[1] + Iv[3 * a + 2] * rn[2]);
    return 1.0 / s.mass + q;
}

double contact_vn(const sph_rigid_desc &s, const double r[3], const double n[3]) {
    double w[3];
    cross3(s.omega, r, w);
    return (s.vel[0] + w[0]) * n[0] + (s.vel[1] + w[1]) * n[1] + (s.vel[2] + w[2]) * n[2];
}

void contact_impulse(sph_rigid_desc &s, const double *Iv, const double r[3], const double n[3], double lam) {
    double rn[3];
    cross3(r, n, rn);
    for (int a = 0; a < 3; ++a) {
        s.vel[a] += lam * n[a] / s.mass;
        s.omega[a] += lam * (Iv[3 * a] * rn[0] + Iv[3 * a + 1] * rn[1] + Iv[3 * a + 2] * rn[2]);
    }
}
}  // namespace

void rigid_contact(sph_ctx *c, double dt, std::vector<sph_rigid_desc> &bs) {
    const int nr = c->nr;
    const double s2 = 2.0 * c->P.r;
    std::vector<std::vector<double>> P(nr);
    std::vector<double> Iv(9 * (size_t)nr, 0.0), reach(nr, 0.0);
    for (int b = 0; b < nr; ++b) {
        double R[9];
        quat_to_R(bs[b].quat, R);
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < 3; ++q)
                for (int k = 0; k < 3; ++k) Iv[9 * b + 3 * a + q] += R[3 * a + k] / bs[b].inertia[k] * R[3 * q + k];
        const std::vector<double> &pts = c->body_points[b];
        P[b].resize(pts.size());
        for (size_t k = 0; k + 2 < pts.size(); k += 3) {
            const double *l = &pts[k];
            for (int a = 0; a < 3; ++a)
                P[b][k + a] = bs[b].com[a] + (R[3 * a] * l[0] + R[3 * a + 1] * l[1] + R[3 * a + 2] * l[2]);
            reach[b] = std::max(reach[b], std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]));
        }
    }
    std::vector<Contact> cs;
    std::vector<std::vector<Contact>> pair_contacts((size_t)nr * nr);
    for (int b = 0; b < nr; ++b)
        for (size_t k = 0; k + 2 < P[b].size(); k += 3)
            for (int a = 0; a < 3; ++a)
                for (int side = 0; side < 2; ++side) {
                    const double plane = side == 0 ? c->P.domain_min[a] + c->P.r : c->P.domain_max[a] - c->P.r;
                    const double g = side == 0 ? P[b][k + a] - plane : plane - P[b][k + a];
                    if (g >= s2) continue;
                    Contact t{};
                    t.a = b;
                    t.b = -1;
                    t.n[a] = side == 0 ? 1.0 : -1.0;
                    for (int q = 0; q < 3; ++q) t.ra[q] = P[b][k + q] - bs[b].com[q];
                    t.bias = -g / dt;
                    t.K = contact_inv_mass(bs[b], &Iv[9 * b], t.ra, t.n);
                    cs.push_back(t);
                }
    // Body pairs.  Two points closer than 2s differ by less than the cell
    // width (a hair over 2s, against rounding) on every axis, so only a's
    // points inside b's bounding box widened by a cell, and b's points inside
    // a's widened box, can touch.  b's points there are binned into a dense
    // grid of such cells (counting sort, ascending index within a cell); each
    // of a's points takes the candidates of its 27 cells in ascending index,
    // so the contacts come in the order of a plain double loop over (k, j).
    const double cell = 2.0 * s2 * (1.0 + 1e-9);
    std::vector<double> box(6 * (size_t)nr);
    for (int b = 0; b < nr; ++b) {
        for (int q = 0; q < 3; ++q) {
            box[6 * b + q] = 1e300;
            box[6 * b + 3 + q] = -1e300;
        }
        for (size_t j = 0; j + 2 < P[b].size(); j += 3)
            for (int q = 0; q < 3; ++q) {
                box[6 * b + q] = std::min(box[6 * b + q], P[b][j + q] - cell);
                box[6 * b + 3 + q] = std::max(box[6 * b + 3 + q], P[b][j + q] + cell);
            }
    }
    auto in_box = [&](int b, const double *x) {
        for (int q = 0; q < 3; ++q)
            if (!(x[q] >= box[6 * b + q] && x[q] <= box[6 * b + 3 + q])) return false;
        return true;
    };
    std::vector<uint32_t> near_b, cstart, cidx, cand;
    for (int a = 0; a < nr; ++a)
        for (int b = a + 1; b < nr; ++b) {
            double dc = 0.0;
            for (int q = 0; q < 3; ++q) dc += (bs[a].com[q] - bs[b].com[q]) * (bs[a].com[q] - bs[b].com[q]);
            if (std::sqrt(dc) >= reach[a] + reach[b] + 2.0 * s2) continue;
            // b's points that may touch a, binned over a's widened box
            near_b.clear();
            for (size_t j = 0; j + 2 < P[b].size(); j += 3)
                if (in_box(a, &P[b][j])) near_b.push_back((uint32_t)j);
            if (near_b.empty()) continue;
            // the grid spans the overlap of the two widened boxes, which holds
            // every point either side keeps; a body many cells across in
            // every direction would make it too large: then every kept point
            // of b is a candidate (the same contacts, found more slowly)
            double o[3], ext[3];
            for (int q = 0; q < 3; ++q) {
                o[q] = std::max(box[6 * a + q], box[6 * b + q]);
                ext[q] = std::min(box[6 * a + 3 + q], box[6 * b + 3 + q]) - o[q];
            }
            const bool gridded = ext[0] < 64.0 * cell && ext[1] < 64.0 * cell && ext[2] < 64.0 * cell;
            int64_t dim[3] = {1, 1, 1};
            if (gridded)
                for (int q = 0; q < 3; ++q) dim[q] = std::max<int64_t>((int64_t)std::floor(ext[q] / cell) + 1, 1);
            auto coord = [&](const double *x, int q) {
                if (!gridded) return (int64_t)0;
                const int64_t v = (int64_t)std::floor((x[q] - o[q]) / cell);
                return std::min<int64_t>(std::max<int64_t>(v, 0), dim[q] - 1);
            };
            const int64_t ncell = dim[0] * dim[1] * dim[2];
            cstart.assign((size_t)ncell + 1, 0u);
            for (const uint32_t j : near_b)
                ++cstart[(size_t)((coord(&P[b][j], 2) * dim[1] + coord(&P[b][j], 1)) * dim[0] + coord(&P[b][j], 0)) + 1];
            for (int64_t t = 0; t < ncell; ++t) cstart[(size_t)t + 1] += cstart[(size_t)t];
            cidx.resize(near_b.size());
            {
                std::vector<uint32_t> fill(cstart.begin(), cstart.end() - 1);
                for (const uint32_t j : near_b) {
                    const size_t t = (size_t)((coord(&P[b][j], 2) * dim[1] + coord(&P[b][j], 1)) * dim[0] +
                                              coord(&P[b][j], 0));
                    cidx[fill[t]++] = j;
                }
            }
            for (size_t k = 0; k + 2 < P[a].size(); k += 3) {
                if (!in_box(b, &P[a][k])) continue;
                const int64_t cx = coord(&P[a][k], 0), cy = coord(&P[a][k], 1), cz = coord(&P[a][k], 2);
                cand.clear();
                for (int64_t z = std::max<int64_t>(cz - 1, 0); z <= std::min(cz + 1, dim[2] - 1); ++z)
                    for (int64_t y = std::max<int64_t>(cy - 1, 0); y <= std::min(cy + 1, dim[1] - 1); ++y)
                        for (int64_t x = std::max<int64_t>(cx - 1, 0); x <= std::min(cx + 1, dim[0] - 1); ++x) {
                            const size_t t = (size_t)((z * dim[1] + y) * dim[0] + x);
                            cand.insert(cand.end(), cidx.begin() + cstart[t], cidx.begin() + cstart[t + 1]);
                        }
                std::sort(cand.begin(), cand.end());
                for (const uint32_t j : cand) {
                    double d[3], dd = 0.0;
                    for (int q = 0; q < 3; ++q) {
                        d[q] = P[a][k + q] - P[b][j + q];
                        dd += d[q] * d[q];
                    }
                    dd = std::sqrt(dd);
                    if (!(dd < 2.0 * s2) || dd == 0.0) continue;
                    Contact t{};
                    t.a = a;
                    t.b = b;
                    for (int q = 0; q < 3; ++q) {
                        t.n[q] = d[q] / dd;
                        t.ra[q] = P[a][k + q] - bs[a].com[q];
                        t.rb[q] = P[b][j + q] - bs[b].com[q];
                    }
                    t.bias = -(dd - s2) / dt;
                    t.K = contact_inv_mass(bs[a], &Iv[9 * a], t.ra, t.n) + contact_inv_mass(bs[b], &Iv[9 * b], t.rb, t.n);
                    pair_contacts[(size_t)a * nr + b].push_back(t);
                }
            }
        }
    // pairs in the order a < b, a outer
    for (int a = 0; a < nr; ++a)
        for (int b = a + 1; b < nr; ++b) {
            std::vector<Contact> &v = pair_contacts[(size_t)a * nr + b];
            cs.insert(cs.end(), v.begin(), v.end());
        }
    for (int sweep = 0; sweep < 30; ++sweep)
        for (Contact &t : cs) {
            double vn = contact_vn(bs[t.a], t.ra, t.n);
            if (t.b >= 0) vn -= contact_vn(bs[t.b], t.rb, t.n);
            const double lam = std::max(0.0, t.lam + (t.bias - vn) / t.K);
            const double dl = lam - t.lam;
            t.lam = lam;
            if (dl == 0.0) continue;
            contact_impulse(bs[t.a], &Iv[9 * t.a], t.ra, t.n, dl);
            if (t.b >= 0) contact_impulse(bs[t.b], &Iv[9 * t.b], t.rb, t.n, -dl);
        }
}

// Newton-Euler in FP64 with the world inertia R diag(I) R^T for every body;
// then rigid contact on the new velocities (or, without it, the tank-contact
// stand-in after the pose moves: push the body back inside [min + r, max - r]
// along each axis and drop the velocity component into the wall).
// advance_velocity false (strong coupling): the velocities were advanced
// during the step, only contact and the pose remain.
void rigid_integrate(sph_ctx *c, double dt, bool advance_velocity) {
    const double *gr = c->P.gravity;
    std::vector<sph_rigid_desc> bs(c->rigid.begin(), c->rigid.begin() + c->nr);
    for (int b = 0; b < c->nr && advance_velocity; ++b) {
        sph_rigid_desc &s = bs[b];
        double R[9], Iw[9], Iwinv[9];
        quat_to_R(s.quat, R);
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < 3; ++q) {
                Iw[3 * a + q] = 0.0;
                Iwinv[3 * a + q] = 0.0;
                for (int k = 0; k < 3; ++k) {
                    Iw[3 * a + q] += R[3 * a + k] * s.inertia[k] * R[3 * q + k];
                    Iwinv[3 * a + q] += R[3 * a + k] / s.inertia[k] * R[3 * q + k];
                }
            }
        for (int a = 0; a < 3; ++a) s.vel[a] += dt * (c->force[3 * b + a] / s.mass + gr[a]);
        double Lw[3], gyro[3], rhs[3];
        for (int a = 0; a < 3; ++a)
            Lw[a] = Iw[3 * a] * s.omega[0] + Iw[3 * a + 1] * s.omega[1] + Iw[3 * a + 2] * s.omega[2];
        cross3(s.omega, Lw, gyro);
        for (int a = 0; a < 3; ++a) rhs[a] = c->torque[3 * b + a] - gyro[a];
        for (int a = 0; a < 3; ++a)
            s.omega[a] += dt * (Iwinv[3 * a] * rhs[0] + Iwinv[3 * a + 1] * rhs[1] + Iwinv[3 * a + 2] * rhs[2]);
    }
    if (c->P.rigid_contact == 1) rigid_contact(c, dt, bs);
    for (int b = 0; b < c->nr; ++b) {
        sph_rigid_desc s = bs[b];
        double R[9];
        for (int a = 0; a < 3; ++a) s.com[a] += dt * s.vel[a];
        {
            double qw = s.quat[0], qx = s.quat[1], qy = s.quat[2], qz = s.quat[3];
            const double ox = s.omega[0], oy = s.omega[1], oz = s.omega[2];
            const double dw = -(ox * qx + oy * qy + oz * qz);
            const double dx = ox * qw + (oy * qz - oz * qy);
            const double dy = oy * qw + (oz * qx - ox * qz);
            const double dz = oz * qw + (ox * qy - oy * qx);
            qw += 0.5 * dt * dw; qx += 0.5 * dt * dx; qy += 0.5 * dt * dy; qz += 0.5 * dt * dz;
            const double nq = std::sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            s.quat[0] = qw / nq; s.quat[1] = qx / nq; s.quat[2] = qy / nq; s.quat[3] = qz / nq;
        }
        if (c->P.rigid_contact != 1) {
            quat_to_R(s.quat, R);
            const std::vector<double> &pts = c->body_points[b];
            for (int a = 0; a < 3; ++a) {
                double lo = 1e300, hi = -1e300;
                for (size_t k = 0; k + 2 < pts.size(); k += 3) {
                    const double *l = &pts[k];
                    const double xa = s.com[a] + (R[3 * a] * l[0] + R[3 * a + 1] * l[1] + R[3 * a + 2] * l[2]);
                    lo = std::min(lo, xa);
                    hi = std::max(hi, xa);
                }
                const double wl = c->P.domain_min[a] + c->P.r, wh = c->P.domain_max[a] - c->P.r;
                if (lo < wl) {
                    s.com[a] += wl - lo;
                    if (s.vel[a] < 0.0) s.vel[a] = 0.0;
                } else if (hi > wh) {
                    s.com[a] -= hi - wh;
                    if (s.vel[a] > 0.0) s.vel[a] = 0.0;
                }
            }
        }
        c->rigid[b] = s;
    }
}

// ---- the neighbour pipeline ------------------------------------------------
int sort_fluid(sph_ctx *c) {
    hipStream_t s = c->stream;
    HIP_TRY(c, sph::launch_fill_u32(c->count, c->ncell, 0u, s));
    HIP_TRY(c, sph::launch_keys_hist(c->x, c->nf, c->g, c->key, c->slot, c->count, s));
    HIP_TRY(c, sph::launch_exclusive_scan(c->count, c->ncell, c->start_f, c->scan_part, s));
    HIP_TRY(c, sph::launch_scatter(c->key, c->slot, c->start_f, c->nf, c->src, s));
    HIP_TRY(c, sph::launch_cell_sort(c->start_f, c->ncell, c->src, c->id, c->flags, s));
    HIP_TRY(c, sph::launch_gather_fluid(c->src, c->nf, c->x, c->v, c->K, c->Kv, c->rho, c->id, c->dvisc, c->x2, c->v2,
                                        c->K2, c->Kv2, c->rho2, c->id2, c->dvisc2, s));
    std::swap(c->dvisc, c->dvisc2);
    std::swap(c->rho, c->rho2);
    std::swap(c->x, c->x2);
    std::swap(c->v, c->v2);
    std::swap(c->K, c->K2);
    std::swap(c->Kv, c->Kv2);
    std::swap(c->id, c->id2);
    return SPH_OK;
}

int sort_boundary(sph_ctx *c) {
    hipStream_t s = c->stream;
    HIP_TRY(c, sph::launch_fill_u32(c->count, c->ncell, 0u, s));
    HIP_TRY(c, sph::launch_keys_hist(c->xb, c->nb, c->g, c->bkey, c->bslot, c->count, s));
    HIP_TRY(c, sph::launch_exclusive_scan(c->count, c->ncell, c->start_b, c->scan_part, s));
    HIP_TRY(c, sph::launch_scatter(c->bkey, c->bslot, c->start_b, c->nb, c->bsrc, s));
    HIP_TRY(c, sph::launch_cell_sort(c->start_b, c->ncell, c->bsrc, c->bid, c->flags, s));
    HIP_TRY(c, sph::launch_gather_boundary(c->bsrc, c->nb, c->xb, c->vb, c->bid, c->xb2, c->vb2, c->bid2, s));
    std::swap(c->xb, c->xb2);
    std::swap(c->vb, c->vb2);
    std::swap(c->bid, c->bid2);
    HIP_TRY(c, sph::launch_boundary_psi(c->xb, c->nb, c->start_b, c->g, c->kc, s));
    return SPH_OK;
}

// algorithmic bytes of reading every neighbour-list entry once (4 B each)
double list_bytes(const sph_ctx *c) { return 4.0 * c->nbr_sum; }
double fluid_list_bytes(const sph_ctx *c) { return 4.0 * c->nbr_sum_f; }

// The neighbour pipeline in two halves: build_queue launches the sorts and
// the list build, build_check reads their status (capacity flags, neighbour
// statistics) once the stream has passed them.
int build_queue(sph_ctx *c) {
    hipStream_t s = c->stream;
    // the sort below replaces id2 and the previous counts: the last step's
    // output order moves there, or, if it is there already, is saved first
    if (c->out_order == sph_ctx::OutOrder::Prev) {
        const size_t n4 = sizeof(int32_t) * (size_t)c->nf;
        HIP_TRY(c, hipMemcpyAsync(c->id_out, c->id2, n4, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(c->ncnt_out, c->ncnt2, n4, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(c->bcnt_out, c->bcnt2, n4, hipMemcpyDeviceToDevice, s));
        c->out_order = sph_ctx::OutOrder::Saved;
    } else if (c->out_order == sph_ctx::OutOrder::Cur) {
        c->out_order = sph_ctx::OutOrder::Prev;
    }
    HIP_TRY(c, sph::launch_fill_u32(c->flags, 1, 0u, s));
    if (c->boundary_dirty) {
        ProfScope ps(c, "sort", 0.0);
        int rc = sort_boundary(c);
        if (rc) return rc;
        c->boundary_dirty = false;
    }
    {
        ProfScope ps(c, "sort", (16.0 + 72.0) * c->nf);   // histogram, scan and scatter ~16 B, reorder 36 + 36
        int rc = sort_fluid(c);
        if (rc) return rc;
    }
    std::swap(c->ncnt, c->ncnt2);   // keep the previous build's counts
    std::swap(c->bcnt, c->bcnt2);
    {
        ProfScope ps(c, "nbr_build", 16.0 * c->nf + list_bytes(c));   // x in, count out, lists written
        HIP_TRY(c, sph::launch_nbr_build(c->x, c->nf, c->xb, c->start_f, c->start_b, c->g, c->nlist, c->ncnt, c->capf,
                                         c->blist, c->bcnt, c->capb, c->flags, c->nstat_part, c->hs_dev, s));
    }
    return SPH_OK;
}

int build_check(sph_ctx *c) {
    const sph::HostStatus &hs = *c->hs;
    c->sorted_once = true;
    if (hs.flags & 2u) {
        c->nbr_fresh = false;
        return fail(c, SPH_ERR_CAPACITY, "more than 4096 particles in one grid cell");
    }
    if (hs.flags & 1u) {
        c->nbr_fresh = false;
        return fail(c, SPH_ERR_CAPACITY, "neighbour list capacity exceeded (max_neighbors / max_boundary_neighbors)");
    }
    for (int f = 0; f < sph::kNStats; ++f) c->nstats[f] = hs.nstats[f];
    c->nbr_sum = (double)hs.nstats[2];
    c->nbr_sum_f = (double)hs.nstats[3];
    c->nbr_fresh = true;
    return SPH_OK;
}

int build(sph_ctx *c) {
    c->build_ahead = false;   // an explicit build replaces one queued ahead
    int rc = build_queue(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return build_check(c);
}

// go (nullable): skip the pass on the device once the solve needs no more
// iterations.
int pressure_pass(sph_ctx *c, float *Kacc, float *klast, float dt, const int32_t *go) {
    ProfScope ps(c, "pressure_update", 52.0 * c->nf + list_bytes(c));   // x, v, kappa in; v, K out
    HIP_TRY(c, sph::launch_pressure_update(c->nf, c->x, c->v, c->kappa, Kacc, klast, c->nlist, c->ncnt, c->xb,
                                           c->blist, c->bcnt, c->kc, dt, go, c->stream));
    return SPH_OK;
}

// Strong coupling: the reaction of the pressure pass just queued (kappa/rho =
// scale x.w) moves the bodies at once and refreshes their boundary
// velocities (go: the solve's control block, or null).
int couple_pass(sph_ctx *c, float dt, float scale, const int32_t *go) {
    if (!c->strong) return SPH_OK;
    HIP_TRY(c, sph::launch_rigid_couple(c->nf, c->x, c->blist, c->bcnt, c->xb, c->vb, c->bid, c->blocal, c->kc, c->nr,
                                        c->com_dev, c->nb, c->red_part, scale, dt, go, c->dyn, c->poses, c->ft,
                                        c->hs_dev, c->stream));
    return SPH_OK;
}

// The predict pass and its finish (the timing record covers the pass only).
int predict_pass(sph_ctx *c, int mode, float dt, bool first, const sph::SolveCtl &init) {
    float *dout = nullptr;   // the learned start's divergence feature comes from the density pass
    int nparts = 0;
    {
        // x and v (plus rho in the density solve) in, kappa out
        ProfScope ps(c, "predict", (mode == 0 ? 32.0 : 36.0) * c->nf + list_bytes(c));
        HIP_TRY(c, sph::launch_predict(mode, c->nf, c->x, c->v, c->rho, c->alpha, c->kappa, c->nlist, c->ncnt,
                                       c->xb, c->vb_moving ? c->vb : nullptr, c->blist, c->bcnt, c->kc, dt,
                                       c->red_part, c->ctl, first,
                                       dout, &nparts, c->stream));
    }
    HIP_TRY(c, sph::launch_solve_finish(c->red_part, nparts, c->ctl, first, init, c->hs_dev, c->stream));
    return SPH_OK;
}

// Control block a solve starts from: err = scale * (sum of the clamped
// deviations), the mean of Algorithm 2 (dt/rho0 for the divergence).
sph::SolveCtl solve_init(const sph_ctx *c, int mode, float dt, int32_t forced, double eta) {
    const double N = (double)std::max<int64_t>(c->nf, 1);
    sph::SolveCtl init{};
    init.scale = mode == 0 ? (double)dt / c->P.rho0 / N : 1.0 / (c->P.rho0 * N);
    init.eta = eta;
    init.forced = forced;
    init.max_iters = c->P.max_iters;
    init.go = 1;
    if (mode == 1 && c->P.eta_density_max > 0.0) {   // the density solve may bound the largest deviation too
        init.eta_max = c->P.eta_density_max;
        init.max_scale = 1.0 / c->P.rho0;
    }
    return init;
}

// The iterations of a Jacobi solve whose first predict pass and finish are
// queued: stop when err <= eta, or after max_iters, or after exactly
// `forced` iterations when forced >= 0.  The stop rule runs on the device
// (SolveCtl): the host queues iterations in batches (the first of
// first_batch) and reads the control block once per batch; passes of
// iterations past the stop do nothing.  tail (nullable) is queued after
// every batch, before the host waits: work that runs only once the solve
// has stopped (it reads the control block's go flag on the device).
int jacobi_iterate(sph_ctx *c, int mode, float dt, float *Kacc, float *klast, const sph::SolveCtl &init,
                   int32_t first_batch, int32_t *iters, double *err_out,
                   const std::function<int()> *tail = nullptr) {
    hipStream_t s = c->stream;
    const int32_t cap = init.forced >= 0 ? init.forced : std::max(init.max_iters, 0);
    const size_t mark = c->prof_pending.size();
    int32_t queued = 0;
    int32_t batch = std::min(first_batch, cap);
    sph::SolveCtl h{};
    for (;;) {
        for (int32_t k = 0; k < batch; ++k) {
            int rc = pressure_pass(c, Kacc, klast, dt, &c->ctl->go);
            if (rc) return rc;
            if ((rc = couple_pass(c, dt, 1.0f, &c->ctl->go))) return rc;
            rc = predict_pass(c, mode, dt, false, init);
            if (rc) return rc;
        }
        queued += batch;
        if (tail) {
            const int rc = (*tail)();
            if (rc) return rc;
        }
        HIP_TRY(c, hipStreamSynchronize(s));
        h = c->hs->solve;
        if (!h.go || queued >= cap) break;
        batch = std::min<int32_t>(queued < 2 ? 1 : 2, cap - queued);
    }
    // drop the timing records of queued passes that did nothing
    if (c->prof && c->prof_pending.size() > mark) {
        // records per iteration: its pressure and predict passes, as far as
        // the profile records them
        const size_t per_iter = (c->prof_only.empty() || c->prof_only == "pressure_update" ? 1 : 0) +
                                (c->prof_only.empty() || c->prof_only == "predict" ? 1 : 0);
        const size_t keep = mark + per_iter * (size_t)h.iters;
        for (size_t q = keep; q < c->prof_pending.size(); ++q) {
            c->event_pool.push_back(c->prof_pending[q].a);
            c->event_pool.push_back(c->prof_pending[q].b);
        }
        if (keep < c->prof_pending.size()) c->prof_pending.resize(keep);
    }
    c->last_iters[mode] = h.iters;
    if (mode == 1) c->last_err_max = h.err_max;
    *iters = h.iters;
    *err_out = h.err;
    return SPH_OK;
}

// One Jacobi solve (Algorithm 2): the first predict pass (the error of the
// starting state), then the iterations, the first batch sized by the
// previous step's count for this solve.
int jacobi_solve(sph_ctx *c, int mode, float dt, float *Kacc, float *klast, int32_t forced, double eta,
                 int32_t *iters, double *err_out, const std::function<int()> *tail = nullptr) {
    const sph::SolveCtl init = solve_init(c, mode, dt, forced, eta);
    int rc = predict_pass(c, mode, dt, true, init);
    if (rc) return rc;
    return jacobi_iterate(c, mode, dt, Kacc, klast, init, c->last_iters[mode], iters, err_out, tail);
}

hipError_t visc_matvec(sph_ctx *c, const float4 *p, float4 *Mp, float dt, float mu, const int32_t *go,
                       double *partials) {
    return sph::launch_visc_matvec(c->nf, c->x, p, Mp, c->nlist, c->ncnt, c->kc, dt, mu, go, partials, c->stream);
}

// WCSPH equation of state (Sec. 3.4.1): kappa = p/rho, x.w = kappa/rho, K = 0,
// and the mean compression of rho as the reported error (read by the host
// after its next synchronisation); the pressure pass follows, on its own or
// inside the non-pressure pass.
int wcsph_eos(sph_ctx *c) {
    hipStream_t s = c->stream;
    int nparts = 0;
    {
        ProfScope ps(c, "eos", 16.0 * c->nf);   // rho in; kappa, K, x.w out
        HIP_TRY(c, sph::launch_eos(c->nf, c->x, c->rho, c->kappa, c->K, c->kc, (float)c->P.wcsph_k,
                                   (float)c->P.wcsph_gamma, c->red_part, &nparts, s));
    }
    sph::SolveCtl init{};
    init.scale = 1.0 / (c->P.rho0 * (double)std::max<int64_t>(c->nf, 1));
    init.eta = c->P.eta_density;
    init.forced = 0;   // no iterations: the finish only records the error
    HIP_TRY(c, sph::launch_solve_finish(c->red_part, nparts, c->ctl, true, init, c->hs_dev, s));
    return SPH_OK;
}

// Implicit viscosity (Eqs. 16-19): CG with block-Jacobi preconditioner on
// (I - dt A) v* = v~ from x0 = v~ + cg_warm_factor (the previous step's
// correction v* - v~), stop at |r| <= tol |b|.  Dot products FP64.  The stop
// rule runs on the device as in jacobi_solve: iterations are queued in
// batches and the host reads the control block once per batch.  An iteration
// is two kernels, the mat-vec of the preconditioned residual (with the u.w
// sums) and the single-reduction update (k_cg_update), whose control blocks
// and update sums alternate between two slots by iteration parity.
int implicit_viscosity(sph_ctx *c, float dt, int32_t *iters, double *resid) {
    hipStream_t s = c->stream;
    const int64_t nf = c->nf;
    *iters = 0;
    *resid = 0.0;
    if (nf == 0) return SPH_OK;
    const float mu = (float)(c->P.visc * c->P.rho0);
    HIP_TRY(c, sph::launch_cg_start(nf, c->v, c->dvisc, c->cg_b, c->v2, dt, (float)c->P.gravity[0],
                                    (float)c->P.gravity[1], (float)c->P.gravity[2], (float)c->P.cg_warm_factor, s));
    {
        ProfScope ps(c, "visc", 60.0 * nf + fluid_list_bytes(c));
        HIP_TRY(c, sph::launch_visc_precond(nf, c->x, c->rho, c->nlist, c->ncnt, c->kc, dt, mu, c->Pinv, s));
    }
    {
        ProfScope ps(c, "visc", 48.0 * nf + fluid_list_bytes(c));
        HIP_TRY(c, visc_matvec(c, c->v2, c->cg_Ap, dt, mu, nullptr, nullptr));
    }
    const int npap = sph::visc_matvec_parts(nf);
    const int64_t nred = (int64_t)sph::reduction_blocks(nf);
    double *uw = c->cg_part, *upd[2] = {c->cg_part + npap, c->cg_part + npap + 2 * nred};
    // the set-up's three sums per workgroup fit the two update slots, read
    // by its own finish before the first update writes there
    HIP_TRY(c, sph::launch_cg_setup(nf, c->cg_b, c->cg_Ap, c->Pinv, c->cg_r, c->cg_z, c->cg_p, upd[0], &c->cgc[0],
                                    c->P.cg_tol, c->P.cg_max_iters, c->hs_dev, s));
    const int32_t cap = std::max(c->P.cg_max_iters, 0);
    const size_t mark = c->prof_pending.size();
    // one mat-vec more than updates: the update after the last one finds the
    // residual converged and stops
    int32_t queued = 0, batch = std::min(std::max(c->last_cg, 1) + 1, cap + 1);
    for (;;) {
        for (int32_t k = 0; k < batch; ++k) {
            const int32_t it = queued + k;
            const int par = it & 1;
            {
                ProfScope ps(c, "visc", 48.0 * nf + fluid_list_bytes(c));
                HIP_TRY(c, visc_matvec(c, c->cg_z, c->cg_Ap, dt, mu, &c->cgc[par].go, uw));
            }
            HIP_TRY(c, sph::launch_cg_iteration(nf, c->v2, c->cg_r, c->cg_z, c->cg_p, c->cg_s, c->cg_Ap, c->Pinv,
                                                &c->cgc[par], &c->cgc[par ^ 1], upd[par ^ 1], uw, npap, upd[par],
                                                c->hs_dev, it == 0, s));
        }
        queued += batch;
        HIP_TRY(c, hipStreamSynchronize(s));
        if (!c->hs->cg.go || queued > cap) break;
        batch = std::min<int32_t>(4, cap + 1 - queued);
    }
    const sph::CgCtl h = c->hs->cg;
    // drop the timing records of queued mat-vecs that did nothing
    if (c->prof && c->prof_pending.size() > mark) {
        const size_t keep = mark + (c->prof_only.empty() || c->prof_only == "visc" ? (size_t)h.iters : 0);
        for (size_t q = keep; q < c->prof_pending.size(); ++q) {
            c->event_pool.push_back(c->prof_pending[q].a);
            c->event_pool.push_back(c->prof_pending[q].b);
        }
        if (keep < c->prof_pending.size()) c->prof_pending.resize(keep);
    }
    c->last_cg = h.iters;
    const double bnorm = h.bnorm, rnorm = std::sqrt(h.rr);
    *iters = h.iters;
    *resid = bnorm > 0 ? rnorm / bnorm : rnorm;
    HIP_TRY(c, sph::launch_visc_correction(nf, c->v2, c->cg_b, c->dvisc, s));
    std::swap(c->v, c->v2);
    return SPH_OK;
}

int step_impl(sph_ctx *c, sph_step_stats *st) {
    hipStream_t s = c->stream;
    // 0. neighbours: with auto_rebuild the build is queued here and its status
    //    read only after the density pass is queued too, so the device runs
    //    that pass while the host waits
    const bool rebuild = !c->nbr_fresh;
    if (rebuild && !c->build_ahead) {
        if (!c->P.auto_rebuild) return fail(c, SPH_ERR_STATE, "sph_step needs fresh neighbours (sph_build_neighbors)");
        int rc = build_queue(c);
        if (rc) return rc;
        HIP_TRY(c, hipEventRecord(c->build_done, s));
    }
    c->build_ahead = false;
    const int64_t nf = c->nf;
    const bool dfsph = c->P.solver == SPH_SOLVER_DFSPH;
    const bool pcisph = c->P.solver == SPH_SOLVER_PCISPH;
    const bool ppe = dfsph || pcisph;   // iterative density solve
    const bool warm = ppe && c->warm_mode != SPH_WARM_ZERO;
    const float wf = warm ? (float)c->P.warm_factor : 0.0f;
    const bool learned = dfsph && c->warm_mode == SPH_WARM_LEARNED && c->mlp != nullptr;
    const bool tracing = dfsph && c->trace_feat != nullptr && c->trace_rows + nf <= c->trace_cap;
    c->want_d = learned || tracing;
    // strong coupling: the bodies' mass and world inertia for this step (the
    // pose stays until the step's end), the summed reaction cleared
    c->strong = c->P.rigid_coupling == 1 && c->nr > 0;
    if (c->strong) {
        std::vector<sph::BodyDyn> dyn(c->nr);
        for (int b = 0; b < c->nr; ++b) {
            const sph_rigid_desc &r = c->rigid[b];
            double R[9];
            quat_to_R(r.quat, R);
            dyn[b].mass = r.mass;
            for (int a = 0; a < 3; ++a)
                for (int q = 0; q < 3; ++q) {
                    dyn[b].Iw[3 * a + q] = 0.0;
                    dyn[b].Iwinv[3 * a + q] = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        dyn[b].Iw[3 * a + q] += R[3 * a + k] * r.inertia[k] * R[3 * q + k];
                        dyn[b].Iwinv[3 * a + q] += R[3 * a + k] / r.inertia[k] * R[3 * q + k];
                    }
                }
        }
        HIP_TRY(c, hipMemcpyAsync(c->dyn, dyn.data(), sizeof(sph::BodyDyn) * c->nr, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, sph::launch_fill_u32(reinterpret_cast<uint32_t *>(c->ft), 2 * 6 * sph::kMaxBodies, 0u, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));   // the host copy of dyn is released below
        std::memset(c->hs->rigid, 0, sizeof(c->hs->rigid));
    }

    // 1. time step (fixed, or CFL from the step's input velocities)
    float dt;
    if (c->P.cfl_lambda > 0.0) {
        // max |v|^2 of the step's input velocities: queued at the end of the
        // previous step (vmax_done), else computed now
        if (c->vmax_ready) {
            HIP_TRY(c, hipEventSynchronize(c->vmax_done));
        } else {
            HIP_TRY(c, sph::launch_max_v2(c->v, nf, (uint32_t *)c->red_part, c->hs_dev, s));
            HIP_TRY(c, hipStreamSynchronize(s));
        }
        c->vmax_ready = false;
        float vmax2;
        std::memcpy(&vmax2, &c->hs->vmax_bits, sizeof(float));
        double d = c->P.dt_max;
        if (vmax2 > 0.0f) {
            const double cfl = c->P.cfl_lambda * (2.0 * c->P.r) / std::sqrt((double)vmax2);
            if (cfl < d) d = cfl;
        }
        dt = (float)d;
    } else {
        dt = (float)c->P.dt_max;
    }

    // 2. density, alpha, and (DFSPH) the divergence solve's warm start; for
    //    the learned start (and its trace) also the density change rate of
    //    the input velocity, one of the network's features
    {
        const bool din = dfsph && c->want_d;
        // x in; rho, alpha, the volume out; with the divergence warm start also v in and out
        ProfScope ps(c, "density_alpha",
                     36.0 * nf + list_bytes(c) + (dfsph && warm ? 16.0 * nf : 0.0) + (din ? 20.0 * nf : 0.0));
        HIP_TRY(c, sph::launch_density_alpha(nf, c->x, c->v, din ? c->v2 : c->v, c->nlist, c->ncnt, c->xb,
                                             c->vb_moving ? c->vb : nullptr, c->blist, c->bcnt, c->kc, c->rho,
                                             c->alpha, c->v_in, c->Kv, dt, dfsph ? wf : 0.0f, c->pci_c,
                                             din ? c->dbuf : nullptr, s));
        if (din) std::swap(c->v, c->v2);
    }
    // the divergence warm start's pressure (applied in the density pass) moves the bodies
    if (dfsph && warm) {
        int rc = couple_pass(c, dt, wf, nullptr);
        if (rc) return rc;
    }
    if (rebuild) {
        HIP_TRY(c, hipEventSynchronize(c->build_done));
        int rc = build_check(c);   // a capacity error leaves clamped, in-bounds lists behind
        if (rc) return rc;
    }
    // 3. divergence-free solve (DFSPH).  Its first predict pass reads the v
    //    the explicit non-pressure pass reads too.  When the last two steps'
    //    solves needed no iteration (a settled flow, whose next step rarely
    //    does), that pass takes the check over (fold); should the error call
    //    for iterations after all, they run after it and the non-pressure
    //    pass is queued again.  A flow whose solve alternates between none
    //    and one iteration keeps the check separate.
    const bool implicit = c->P.visc_model == SPH_VISC_IMPLICIT;
    const bool fold = dfsph && !implicit && !tracing && !c->strong && !c->P.separate_div_check &&
                      c->forced_div < 0 && c->div_calm >= 2;
    int32_t iv = 0, id = 0;
    double ev = 0.0, ed = 0.0;
    int rc = SPH_OK;
    if (dfsph && !fold) {
        rc = jacobi_solve(c, 0, dt, c->Kv, nullptr, c->forced_div, c->P.eta_divergence, &iv, &ev);
        if (rc) return rc;
    }
    // strong coupling: the bodies' gravity and gyroscopic term, between the
    // solves as the fluid's non-pressure accelerations
    if (c->strong)
        HIP_TRY(c, sph::launch_rigid_gravity(c->nr, c->nb, c->xb, c->vb, c->bid, c->blocal, c->dyn, c->poses,
                                             c->P.gravity[0], c->P.gravity[1], c->P.gravity[2], dt, s));

    // 4. non-pressure accelerations and the density warm start (or WCSPH's
    //    equation of state).  The warm start's stiffness is set up first: the
    //    previous stiffness, or the MLP's prediction from per-particle
    //    features (density, the divergence left by the divergence-free solve,
    //    neighbour count, previous stiffness, alpha), which also feed the
    //    training trace.  With explicit viscosity one neighbour pass then
    //    applies both v* and that stiffness's pressure.
    int32_t cg_it = 0;
    double cg_res = 0.0;
    const float gx = (float)c->P.gravity[0], gy = (float)c->P.gravity[1], gz = (float)c->P.gravity[2];
    const bool wcsph = c->P.solver == SPH_SOLVER_WCSPH;
    auto warm_setup = [&](float *Ksave) -> int {   // kappa = K0, K = 0, x.w = K0 / rho
        const float alpha_ref = (float)(2.35376 * 4.0 * c->P.r * c->P.r / c->P.rho0);
        if (learned && !tracing) {   // features, network and start in one pass
            ProfScope ps(c, "mlp", 36.0 * nf);
            HIP_TRY(c, sph::launch_mlp_warm_start(c->mlp->packed, nf, c->x, c->rho, c->alpha, c->K, c->kappa, c->ncnt,
                                                  c->bcnt, c->dbuf, c->kc, dt, alpha_ref, Ksave, s));
            return SPH_OK;
        }
        if (learned || tracing) {
            float *feat = tracing ? c->trace_feat + 5 * c->trace_rows : c->feat;
            {
                ProfScope ps(c, "warm_features", 28.0 * nf + 20.0 * nf);
                HIP_TRY(c, sph::launch_features(nf, c->rho, c->alpha, c->K, c->ncnt, c->bcnt, c->dbuf, c->kc, dt,
                                                alpha_ref, feat, s));
            }
            if (learned) {
                {
                    ProfScope ps(c, "mlp", 24.0 * nf);
                    HIP_TRY(c, sph::launch_mlp_forward(c->mlp->packed, feat, nf, c->ybuf, s));
                }
                HIP_TRY(c, sph::launch_warm_learned(nf, c->x, c->rho, c->alpha, c->ybuf, c->K, c->kappa, dt,
                                                    (float)c->P.rho0, s));
                return SPH_OK;
            }
        }
        HIP_TRY(c, sph::launch_warm_setup(nf, c->x, c->rho, c->K, c->kappa, wf, Ksave, s));
        return SPH_OK;
    };
    if (implicit) {
        rc = implicit_viscosity(c, dt, &cg_it, &cg_res);
        if (rc) return rc;
        if (ppe && (rc = warm_setup(nullptr))) return rc;
        if (ppe && warm && (rc = pressure_pass(c, c->K, nullptr, dt, nullptr))) return rc;
        if (ppe && warm && (rc = couple_pass(c, dt, 1.0f, nullptr))) return rc;
        if (wcsph) {
            if ((rc = wcsph_eos(c))) return rc;
            if ((rc = pressure_pass(c, c->K, c->kappa_last, dt, nullptr))) return rc;
            if ((rc = couple_pass(c, dt, 1.0f, nullptr))) return rc;
        }
    } else {
        // the ZERO start only clears K and kappa, inside the pass
        const bool setup_in_pass = ppe && !warm && !(learned || tracing);
        const bool press = (ppe && warm) || wcsph;
        auto nonpressure = [&](bool with_press, const sph::DivCheck *dc, int *nparts) -> int {
            const double walk = (with_press || dc) ? list_bytes(c) : fluid_list_bytes(c);
            // x, v in, v* out; the warm start's pressure adds its 32/12, the folded check the predict's 32
            ProfScope ps(c, "xsph", 40.0 * nf + (with_press ? 44.0 * nf : 0.0) + (dc ? 32.0 * nf : 0.0) + walk);
            HIP_TRY(c, sph::launch_nonpressure(c->P.visc_model, nf, c->x, c->v, c->v2, c->rho, c->nlist, c->ncnt,
                                               c->kc, dt, gx, gy, gz, (float)c->P.visc, c->K, c->kappa, wf,
                                               setup_in_pass, with_press, c->xb, c->blist, c->bcnt,
                                               wcsph ? c->kappa_last : nullptr, dc, nparts, s));
            return SPH_OK;
        };
        if (!fold) {
            if (ppe && !setup_in_pass && (rc = warm_setup(nullptr))) return rc;
            if (wcsph && (rc = wcsph_eos(c))) return rc;
            if ((rc = nonpressure(press, nullptr, nullptr))) return rc;
            std::swap(c->v, c->v2);
            if (press && (rc = couple_pass(c, dt, 1.0f, nullptr))) return rc;
        } else {
            // The start (previous or learned) is set up first (K kept) and
            // the pass applies its pressure as well.
            const bool fold_press = press;
            if (fold_press && (rc = warm_setup(c->K_saved))) return rc;
            const sph::DivCheck dc{c->vb_moving ? c->vb : nullptr, c->alpha, c->div_kvs, nullptr,
                                   c->red_part};
            int nparts = 0;
            if ((rc = nonpressure(fold_press, &dc, &nparts))) return rc;
            const sph::SolveCtl init = solve_init(c, 0, dt, c->forced_div, c->P.eta_divergence);
            HIP_TRY(c, sph::launch_solve_finish(c->red_part, nparts, c->ctl, true, init, c->hs_dev, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            const sph::SolveCtl h = c->hs->solve;
            if (h.go) {   // iterations due: the state the separate check leaves, the solve, the pass again
                if (fold_press)
                    HIP_TRY(c, sph::launch_div_resume(nf, c->x, c->kappa, c->K, c->div_kvs, c->K_saved, s));
                if ((rc = jacobi_iterate(c, 0, dt, c->Kv, nullptr, init, 1, &iv, &ev))) return rc;
                if (ppe && !setup_in_pass && (rc = warm_setup(nullptr))) return rc;
                if ((rc = nonpressure(press, nullptr, nullptr))) return rc;
                std::swap(c->v, c->v2);
            } else {
                c->last_iters[0] = 0;
                iv = 0;
                ev = h.err;
                std::swap(c->v, c->v2);
            }
        }
    }
    // 8 (below) queued behind every batch of the density solve, gated on its
    // stop, so that the device integrates as soon as the solve has stopped
    // instead of after the host has seen it; not with rigid bodies or a
    // trace, whose host work comes in between
    const bool cfl = c->P.cfl_lambda > 0.0;
    const bool early_integrate = ppe && c->nr == 0 && !tracing;
    const std::function<int()> integrate_tail = [&]() -> int {
        HIP_TRY(c, sph::launch_integrate(nf, c->x, c->v, dt, cfl ? (uint32_t *)c->red_part : nullptr, c->hs_dev,
                                         &c->ctl->go, s));
        return SPH_OK;
    };
    if (ppe) {
        // 6. constant-density solve; every pressure pass of it writes the
        //    stiffness it applied to kappa_last, which is zero without one
        rc = jacobi_solve(c, 1, dt, c->K, c->kappa_last, c->forced_dens, c->P.eta_density, &id, &ed,
                          early_integrate ? &integrate_tail : nullptr);
        if (rc) return rc;
        if (id == 0) HIP_TRY(c, sph::launch_fill_f32(c->kappa_last, nf, 0.0f, s));
    } else {
        // 6w. WCSPH: the error the equation-of-state pass recorded
        HIP_TRY(c, hipStreamSynchronize(s));
        ed = c->hs->solve.err;
    }

    if (tracing) {
        HIP_TRY(c, sph::launch_trace_target(nf, c->alpha, c->K, dt, (float)c->P.rho0, c->trace_target + c->trace_rows, s));
        c->trace_rows += nf;
    }
    // 7. rigid bodies: Eq. 14 reaction, FP64 Newton-Euler, new boundary pose
    if (c->nr > 0) {
        // weak coupling: the step's total reaction now; strong: summed pass
        // by pass, the velocities already advanced on the device
        if (!c->strong)
            HIP_TRY(c, sph::launch_rigid_force(nf, c->x, c->rho, c->K, c->Kv, c->blist, c->bcnt, c->xb, c->vb, c->kc,
                                               c->nr, c->com_dev, c->red_part, c->hs_dev, s));
        std::vector<double> fo(6 * c->nr);
        std::vector<sph::BodyPose> pz(c->strong ? c->nr : 0);
        if (c->strong)
            HIP_TRY(c, hipMemcpyAsync(pz.data(), c->poses, sizeof(sph::BodyPose) * c->nr, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        std::memcpy(fo.data(), c->hs->rigid, sizeof(double) * 6 * c->nr);
        for (int b = 0; b < c->nr; ++b)
            for (int a = 0; a < 3; ++a) {
                c->force[3 * b + a] = fo[6 * b + a];
                c->torque[3 * b + a] = fo[6 * b + 3 + a];
                if (c->strong) {
                    c->rigid[b].vel[a] = pz[b].vel[a];
                    c->rigid[b].omega[a] = pz[b].omega[a];
                }
            }
        rigid_integrate(c, (double)dt, !c->strong);
        rc = upload_poses(c);
        if (rc) return rc;
        HIP_TRY(c, sph::launch_rigid_boundary(c->nb, c->xb, c->vb, c->bid, c->blocal, c->poses, s));
        c->boundary_dirty = true;
    }
    // 8. symplectic Euler: v = v*, x += dt v (already done after the density
    //    solve's last batch when early_integrate)
    if (!early_integrate) {
        ProfScope ps(c, "integrate", 44.0 * nf);
        // with a CFL step the pass also reduces the next step's input max |v|^2
        HIP_TRY(c, sph::launch_integrate(nf, c->x, c->v, dt, cfl ? (uint32_t *)c->red_part : nullptr, c->hs_dev,
                                         nullptr, s));
    }
    if (cfl) {   // read after the next step's neighbour build is queued
        HIP_TRY(c, hipEventRecord(c->vmax_done, s));
        c->vmax_ready = true;
    }
    // this step's outputs are in the current order until the next sort
    c->out_order = sph_ctx::OutOrder::Cur;
    // auto_rebuild: the next step's sort and neighbour build go on the stream
    // now, so the device runs them while the host returns and comes back;
    // the next step reads their status after its density pass
    if (c->P.auto_rebuild) {
        int brc = build_queue(c);
        if (brc) return brc;
        HIP_TRY(c, hipEventRecord(c->build_done, s));
        c->build_ahead = true;
    }
    if (dfsph) c->div_calm = iv == 0 ? std::min(c->div_calm + 1, 2) : 0;
    c->nbr_fresh = false;
    c->last_dt = dt;
    c->step_index += 1;
    if (st) {
        st->dt = dt;
        st->iters_div = iv;
        st->iters_dens = id;
        st->err_div = ev;
        st->err_dens = ed;
        st->err_dens_max = c->P.eta_density_max > 0.0 ? c->last_err_max : 0.0;
        st->converged_div = ev <= c->P.eta_divergence;
        st->converged_dens = ed <= c->P.eta_density &&
                             (c->P.eta_density_max <= 0.0 || c->last_err_max <= c->P.eta_density_max);
        st->cg_iters = cg_it;
        st->cg_resid = cg_res;
        st->nbr_min = (int32_t)(c->nstats[0] >= 0xffffffffull ? 0 : c->nstats[0]);
        st->nbr_max = (int32_t)c->nstats[1];
        st->nbr_mean = c->nf ? (double)c->nstats[2] / (double)c->nf : 0.0;
        st->warm_fallback = c->warm_fallback ? 1 : 0;
        st->step_index = c->step_index;
    }
    if (!std::isfinite(ed) || !std::isfinite(ev)) return fail(c, SPH_ERR_NUMERIC, "non-finite solver error");
    return SPH_OK;
}

// PCISPH's delta = 1 / (2 (dt m / rho0)^2 sum_j |gradW_j|^2), summed over the
// neighbours of a particle inside a filled lattice of spacing 2r (where
// sum_j gradW_j = 0), written as the factor c of the density solve's
// kappa_i = (rho*_i - rho0) c / (rho_i dt^2):  c = rho0^2 / (2 m^2 sum_j |gradW_j|^2).
// Host FP64, once per context.
double pcisph_factor(const sph_params &p) {
    const double s = 2.0 * p.r, h = p.h, m = p.rho0 * s * s * s;
    const double k6 = 48.0 / (M_PI * h * h * h * h);   // 6 * 8 / (pi h^3) / h
    const int reach = (int)std::ceil(h / s);
    double g2 = 0.0;
    for (int i = -reach; i <= reach; ++i)
        for (int j = -reach; j <= reach; ++j)
            for (int k = -reach; k <= reach; ++k) {
                const double q = s * std::sqrt((double)(i * i + j * j + k * k)) / h;
                if (q <= 0.0 || q >= 1.0) continue;
                const double slope = q <= 0.5 ? q * (3.0 * q - 2.0) : -(1.0 - q) * (1.0 - q);   // dW/dr / k6
                g2 += (k6 * slope) * (k6 * slope);
            }
    return p.rho0 * p.rho0 / (2.0 * m * m * g2);
}

bool finite3(const float *p, int64_t n) {
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

namespace {
template <typename T>
int d2h(sph_ctx *c, std::vector<T> &h, const T *d, int64_t n) {
    h.resize(std::max<int64_t>(n, 1));
    HIP_TRY(c, hipMemcpyAsync(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, c->stream));
    return SPH_OK;
}
}  // namespace

// ============================================================================ ABI
extern "C" {

const char *sph_strerror(int status) {
    switch (status) {
        case SPH_OK: return "ok";
        case SPH_ERR_INVALID: return "invalid argument";
        case SPH_ERR_OOM: return "out of memory";
        case SPH_ERR_DEVICE: return "HIP error";
        case SPH_ERR_CAPACITY: return "neighbour capacity exceeded";
        case SPH_ERR_STATE: return "call out of order";
        case SPH_ERR_NUMERIC: return "non-finite state";
        default: return "unknown status";
    }
}

const char *sph_last_error(const sph_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

// sph_create, or with count_bytes the device bytes it would allocate (the
// same validation and the same allocation sequence, no memory touched)
static int create_impl(const sph_params *p, const sph_scene *sc, void *hip_stream, sph_ctx **out,
                       int64_t *count_bytes) {
    g_create_error.clear();
    if (!out) return fail(nullptr, SPH_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!p || !sc) return fail(nullptr, SPH_ERR_INVALID, "params or scene is NULL");
    if (!(p->r > 0) || !(p->h > 0) || !(p->rho0 > 0) || !(p->dt_max > 0) || p->max_iters < 0 ||
        p->max_neighbors <= 0 || p->max_boundary_neighbors <= 0 || p->cfl_lambda < 0 || p->warm_factor < 0 ||
        p->visc_model < 0 || p->visc_model > 3 || p->warm_start < 0 || p->warm_start > 2 || p->cg_max_iters < 0 ||
        p->solver < 0 || p->solver > 2 || (p->solver == SPH_SOLVER_WCSPH && !(p->wcsph_k > 0 && p->wcsph_gamma > 0)))
        return fail(nullptr, SPH_ERR_INVALID, "invalid parameter value");
    if (!(p->cg_warm_factor >= 0.0 && p->cg_warm_factor <= 4.0))
        return fail(nullptr, SPH_ERR_INVALID, "cg_warm_factor outside [0, 4]");
    if (p->rigid_coupling != 0 && p->rigid_coupling != 1)
        return fail(nullptr, SPH_ERR_INVALID, "rigid_coupling must be 0 (weak) or 1 (strong)");
    if (p->rigid_contact != 0 && p->rigid_contact != 1)
        return fail(nullptr, SPH_ERR_INVALID, "rigid_contact must be 0 (tank stand-in) or 1 (contact)");
    if (!(p->eta_density_max >= 0.0))
        return fail(nullptr, SPH_ERR_INVALID, "eta_density_max must be >= 0");
    if (!(p->alpha_max_factor >= 0.0 && p->alpha_max_factor <= 1e6))
        return fail(nullptr, SPH_ERR_INVALID, "alpha_max_factor outside [0, 1e6]");
    if (p->separate_div_check != 0 && p->separate_div_check != 1)
        return fail(nullptr, SPH_ERR_INVALID, "separate_div_check must be 0 or 1");
    if (p->solver != SPH_SOLVER_DFSPH && p->warm_start == SPH_WARM_LEARNED)
        return fail(nullptr, SPH_ERR_INVALID, "the learned warm start needs the DFSPH solver");
    for (int a = 0; a < 3; ++a)
        if (!(p->domain_max[a] > p->domain_min[a])) return fail(nullptr, SPH_ERR_INVALID, "empty domain");
    if (sc->n_fluid < 0 || sc->n_boundary < 0 || sc->n_rigid < 0 || sc->n_rigid > sph::kMaxBodies)
        return fail(nullptr, SPH_ERR_INVALID, "invalid scene sizes (at most 16 rigid bodies)");
    if (!count_bytes && ((sc->n_fluid > 0 && !sc->x_fluid) || (sc->n_boundary > 0 && !sc->x_boundary) ||
                         (sc->n_rigid > 0 && (!sc->rigid || !sc->body_of_boundary))))
        return fail(nullptr, SPH_ERR_INVALID, "missing scene array");
    if (!count_bytes && sc->device_arena && sc->device_arena_bytes <= 0)
        return fail(nullptr, SPH_ERR_INVALID, "device_arena given with no bytes");
    if (!count_bytes && sc->device_arena && (uintptr_t)sc->device_arena % 256 != 0)
        return fail(nullptr, SPH_ERR_INVALID, "device_arena must be 256-byte aligned");
    if (sc->n_fluid >= (int64_t)0x7fffffff || sc->n_boundary >= (int64_t)0x7fffffff)
        return fail(nullptr, SPH_ERR_INVALID, "too many particles for 32-bit indices");
    if (!count_bytes) {   // the scene's arrays
        if (sc->n_fluid > 0 && !finite3(sc->x_fluid, sc->n_fluid))
            return fail(nullptr, SPH_ERR_INVALID, "non-finite fluid position");
        if (sc->body_of_boundary)
            for (int64_t k = 0; k < sc->n_boundary; ++k)
                if (sc->body_of_boundary[k] < -1 || sc->body_of_boundary[k] >= sc->n_rigid)
                    return fail(nullptr, SPH_ERR_INVALID, "body_of_boundary out of range");
        for (int b = 0; b < sc->n_rigid; ++b)
            if (!(sc->rigid[b].mass > 0) || !(sc->rigid[b].inertia[0] > 0) || !(sc->rigid[b].inertia[1] > 0) ||
                !(sc->rigid[b].inertia[2] > 0))
                return fail(nullptr, SPH_ERR_INVALID, "rigid body mass and inertia must be positive");
    }

    sph_ctx *c = new (std::nothrow) sph_ctx();
    if (!c) return fail(nullptr, SPH_ERR_OOM, "host allocation failed");
    c->P = *p;
    c->warm_mode = p->warm_start == SPH_WARM_LEARNED ? SPH_WARM_PREVIOUS : p->warm_start;
    c->stream = (hipStream_t)hip_stream;
    c->nf = sc->n_fluid;
    c->nb = sc->n_boundary;
    c->nr = sc->n_rigid;
    c->vb_moving = c->nr > 0;
    c->capf = p->max_neighbors;
    c->capb = p->max_boundary_neighbors;
    (void)hipGetDevice(&c->device);

    // grid: cell fl32(h (1 + 2^-10)), inv fl32(1/cell), origin fl32(min - cell)
    c->cell = (float)(p->h * (1.0 + 1.0 / 1024.0));
    c->g.inv = 1.0f / c->cell;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        c->g.o[a] = (float)(p->domain_min[a] - (double)c->cell);
        c->g.n[a] = (int32_t)std::ceil((p->domain_max[a] - p->domain_min[a]) / (double)c->cell) + 2;
        ncell *= c->g.n[a];
    }
    const float hf = (float)p->h;
    c->g.h2 = hf * hf;
    c->ncell = ncell;
    if (ncell > 16LL * 1024 * 1024) {
        delete c;
        return fail(nullptr, SPH_ERR_INVALID, "grid larger than 16.7M cells");
    }
    // kernel constants
    const double kk = 8.0 / (M_PI * p->h * p->h * p->h);
    c->kc.h = (float)p->h;
    c->kc.inv_h = (float)(1.0 / p->h);
    c->kc.k = (float)kk;
    c->kc.kg = (float)(6.0 * kk / p->h);
    c->kc.m = (float)(p->rho0 * 8.0 * p->r * p->r * p->r);
    c->kc.rho0 = (float)p->rho0;
    c->kc.alpha_max = p->alpha_max_factor > 0.0
                          ? (float)(p->alpha_max_factor * 2.35376 * 4.0 * p->r * p->r / p->rho0)
                          : 0.0f;
    {   // 1e-12 of a bulk lattice particle's sum of |m gradW|^2 (the gradient sum vanishes there)
        const double s = 2.0 * p->r, m = p->rho0 * s * s * s, k6 = 48.0 / (M_PI * p->h * p->h * p->h * p->h);
        const int reach = (int)std::ceil(p->h / s);
        double dsum = 0.0;
        for (int a = -reach; a <= reach; ++a)
            for (int b = -reach; b <= reach; ++b)
                for (int e = -reach; e <= reach; ++e) {
                    const double q = s * std::sqrt((double)(a * a + b * b + e * e)) / p->h;
                    if (q == 0.0 || q >= 1.0) continue;
                    const double fp = q <= 0.5 ? q * (3.0 * q - 2.0) : -(1.0 - q) * (1.0 - q);   // f'(q) / 6
                    const double g = m * k6 * fp;
                    dsum += g * g;
                }
        c->kc.d_min = (float)(1e-12 * dsum);
    }
    if (p->solver == SPH_SOLVER_PCISPH) c->pci_c = (float)pcisph_factor(*p);

    const int64_t nf = c->nf, nb = c->nb;
    const int64_t scan_chunks = (ncell + 4095) / 4096;
    // reductions run over up to four lanes per fluid particle
    const int64_t nred = std::max<int64_t>(sph::reduction_blocks(std::max(4 * nf, nb)), 8);
    int rc = SPH_OK;
    c->counting = count_bytes != nullptr;
    c->arena = count_bytes ? nullptr : (char *)sc->device_arena;
    c->arena_bytes = sc->device_arena_bytes;
#define ALLOC(ptr, n)                       \
    if ((rc = dev_alloc(c, &(ptr), (n)))) { \
        std::string m_ = c->err;            \
        free_all(c);                        \
        delete c;                           \
        return fail(nullptr, rc, m_);       \
    }
    ALLOC(c->x, nf); ALLOC(c->x2, nf); ALLOC(c->v, nf); ALLOC(c->v2, nf); ALLOC(c->v_in, nf);
    ALLOC(c->rho, nf); ALLOC(c->rho2, nf); ALLOC(c->alpha, nf); ALLOC(c->K, nf); ALLOC(c->K2, nf); ALLOC(c->Kv, nf); ALLOC(c->Kv2, nf);
    ALLOC(c->kappa, nf); ALLOC(c->kappa_last, nf); ALLOC(c->id, nf); ALLOC(c->id2, nf);
    ALLOC(c->div_kvs, nf); ALLOC(c->K_saved, nf);
    ALLOC(c->key, nf); ALLOC(c->slot, nf); ALLOC(c->src, nf);
    ALLOC(c->count, ncell); ALLOC(c->start_f, ncell + 1); ALLOC(c->start_b, ncell + 1); ALLOC(c->scan_part, 2 * scan_chunks + 8);
    // 32-bit lists in chunks of four entries (capacity rounded up to a chunk)
    ALLOC(c->nlist, (int64_t)(c->capf + 3) / 4 * 4 * nf); ALLOC(c->ncnt, nf); ALLOC(c->ncnt2, nf);
    ALLOC(c->id_out, nf); ALLOC(c->ncnt_out, nf); ALLOC(c->bcnt_out, nf);
    ALLOC(c->blist, (int64_t)(c->capb + 3) / 4 * 4 * nf); ALLOC(c->bcnt, nf); ALLOC(c->bcnt2, nf);
    ALLOC(c->xb, nb); ALLOC(c->xb2, nb); ALLOC(c->vb, nb); ALLOC(c->vb2, nb); ALLOC(c->bid, nb); ALLOC(c->bid2, nb);
    ALLOC(c->bkey, nb); ALLOC(c->bslot, nb); ALLOC(c->bsrc, nb); ALLOC(c->blocal, 3 * nb);
    ALLOC(c->poses, std::max(1, c->nr)); ALLOC(c->com_dev, 3 * std::max(1, c->nr));
    ALLOC(c->dyn, std::max(1, c->nr)); ALLOC(c->ft, 12 * sph::kMaxBodies);
    ALLOC(c->red_part, nred * 6 * std::max(1, c->nr) + 16); ALLOC(c->scal, 16);
    ALLOC(c->ctl, 1); ALLOC(c->cgc, 2);
    ALLOC(c->flags, 4);
    ALLOC(c->nstat_part, sph::kNStats * nred);
    ALLOC(c->feat, 5 * nf); ALLOC(c->ybuf, nf); ALLOC(c->dbuf, nf);
    if (p->visc_model == SPH_VISC_IMPLICIT) {
        ALLOC(c->Pinv, 3 * nf); ALLOC(c->cg_b, nf); ALLOC(c->cg_r, nf); ALLOC(c->cg_z, nf); ALLOC(c->cg_p, nf);
        ALLOC(c->cg_Ap, nf); ALLOC(c->dvisc, nf); ALLOC(c->dvisc2, nf);
        ALLOC(c->cg_s, nf);
        ALLOC(c->cg_part, sph::visc_matvec_parts(nf) + 4 * (int64_t)sph::reduction_blocks(nf) + 16);
    }
#undef ALLOC
    if (count_bytes) {
        *count_bytes = c->dev_bytes;
        delete c;
        return SPH_OK;
    }
    if (hipHostMalloc((void **)&c->hs, sizeof(sph::HostStatus), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&c->hs_dev, c->hs, 0) != hipSuccess) {
        free_all(c);
        delete c;
        return fail(nullptr, SPH_ERR_OOM, "pinned host allocation failed");
    }
    if (hipEventCreateWithFlags(&c->build_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->vmax_done, hipEventDisableTiming) != hipSuccess) {
        free_all(c);
        delete c;
        return fail(nullptr, SPH_ERR_DEVICE, "event creation failed");
    }
    // upload the scene (original order; the first build sorts it)
    {
        std::vector<float4> hx(std::max<int64_t>(nf, 1)), hv(std::max<int64_t>(nf, 1));
        std::vector<int32_t> hid(std::max<int64_t>(nf, 1));
        for (int64_t i = 0; i < nf; ++i) {
            hx[i] = make_float4(sc->x_fluid[3 * i], sc->x_fluid[3 * i + 1], sc->x_fluid[3 * i + 2], 0.f);
            hv[i] = sc->v_fluid ? make_float4(sc->v_fluid[3 * i], sc->v_fluid[3 * i + 1], sc->v_fluid[3 * i + 2], 0.f)
                                : make_float4(0.f, 0.f, 0.f, 0.f);
            hid[i] = (int32_t)i;
        }
        std::vector<float> zero(std::max<int64_t>(nf, 1), 0.0f);
        // the "previous" density of the first step (its divergence warm start is zero)
        std::vector<float> rho0v(std::max<int64_t>(nf, 1), (float)p->rho0);
        hipStream_t s = c->stream;
        bool ok = hipMemcpyAsync(c->x, hx.data(), sizeof(float4) * nf, hipMemcpyHostToDevice, s) == hipSuccess &&
                  hipMemcpyAsync(c->v, hv.data(), sizeof(float4) * nf, hipMemcpyHostToDevice, s) == hipSuccess &&
                  hipMemcpyAsync(c->id, hid.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice, s) == hipSuccess &&
                  hipMemcpyAsync(c->K, zero.data(), sizeof(float) * nf, hipMemcpyHostToDevice, s) == hipSuccess &&
                  hipMemcpyAsync(c->Kv, zero.data(), sizeof(float) * nf, hipMemcpyHostToDevice, s) == hipSuccess &&
                  hipMemcpyAsync(c->rho, rho0v.data(), sizeof(float) * nf, hipMemcpyHostToDevice, s) == hipSuccess &&
                  (!c->dvisc || hipMemsetAsync(c->dvisc, 0, sizeof(float4) * nf, s) == hipSuccess);
        // boundary: positions, velocities from the body state, body ids, local offsets
        c->rigid.assign(sc->rigid, sc->rigid + c->nr);
        c->force.assign(3 * std::max(1, c->nr), 0.0);
        c->torque.assign(3 * std::max(1, c->nr), 0.0);
        c->local_host.assign(3 * std::max<int64_t>(nb, 1), 0.0);
        c->body_host.assign(std::max<int64_t>(nb, 1), -1);
        std::vector<double> &local = c->local_host;
        std::vector<float4> hxb(std::max<int64_t>(nb, 1)), hvb(std::max<int64_t>(nb, 1));
        std::vector<int32_t> hbid(std::max<int64_t>(nb, 1));
        for (int64_t k = 0; k < nb; ++k) {
            const int32_t b = sc->body_of_boundary ? sc->body_of_boundary[k] : -1;
            c->body_host[k] = b;
            hxb[k] = make_float4(sc->x_boundary[3 * k], sc->x_boundary[3 * k + 1], sc->x_boundary[3 * k + 2], 0.f);
            hvb[k] = make_float4(0.f, 0.f, 0.f, (float)b);
            hbid[k] = (int32_t)k;
            if (b >= 0) {
                const sph_rigid_desc &s = c->rigid[b];
                double R[9], d[3], rr[3], wx[3];
                quat_to_R(s.quat, R);
                for (int a = 0; a < 3; ++a) d[a] = (double)sc->x_boundary[3 * k + a] - s.com[a];
                for (int a = 0; a < 3; ++a) local[3 * k + a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
                for (int a = 0; a < 3; ++a) rr[a] = (double)sc->x_boundary[3 * k + a] - s.com[a];
                cross3(s.omega, rr, wx);
                hvb[k].x = (float)(s.vel[0] + wx[0]);
                hvb[k].y = (float)(s.vel[1] + wx[1]);
                hvb[k].z = (float)(s.vel[2] + wx[2]);
            }
        }
        c->body_points.assign(std::max(1, c->nr), {});
        for (int64_t k = 0; k < nb; ++k)
            if (c->body_host[k] >= 0)
                c->body_points[c->body_host[k]].insert(c->body_points[c->body_host[k]].end(), &local[3 * k],
                                                       &local[3 * k] + 3);
        ok = ok && hipMemcpyAsync(c->xb, hxb.data(), sizeof(float4) * nb, hipMemcpyHostToDevice, s) == hipSuccess &&
             hipMemcpyAsync(c->vb, hvb.data(), sizeof(float4) * nb, hipMemcpyHostToDevice, s) == hipSuccess &&
             hipMemcpyAsync(c->bid, hbid.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s) == hipSuccess &&
             hipMemcpyAsync(c->blocal, local.data(), sizeof(double) * 3 * nb, hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && hipStreamSynchronize(s) == hipSuccess;
        if (!ok) {
            free_all(c);
            delete c;
            return fail(nullptr, SPH_ERR_DEVICE, "scene upload failed");
        }
    }
    if (upload_poses(c) != SPH_OK) {
        std::string m = c->err;
        free_all(c);
        delete c;
        return fail(nullptr, SPH_ERR_DEVICE, m);
    }
    *out = c;
    return SPH_OK;
}

int sph_create(const sph_params *p, const sph_scene *sc, void *hip_stream, sph_ctx **out) {
    return create_impl(p, sc, hip_stream, out, nullptr);
}

int sph_required_bytes(const sph_params *p, const sph_scene *sc, int64_t *bytes) {
    if (!bytes) return fail(nullptr, SPH_ERR_INVALID, "bytes is NULL");
    sph_ctx *unused = nullptr;
    *bytes = 0;
    return create_impl(p, sc, nullptr, &unused, bytes);
}

void sph_destroy(sph_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

int sph_build_neighbors(sph_ctx *c) {
    if (!c) return SPH_ERR_INVALID;
    c->err.clear();
    return build(c);
}

int sph_step(sph_ctx *c, sph_step_stats *st) {
    if (!c) return SPH_ERR_INVALID;
    c->err.clear();
    return step_impl(c, st);
}

int sph_get_info(const sph_ctx *c, sph_info *info) {
    if (!c || !info) return SPH_ERR_INVALID;
    info->n_fluid = c->nf;
    info->n_boundary = c->nb;
    info->n_rigid = c->nr;
    for (int a = 0; a < 3; ++a) {
        info->grid_n[a] = c->g.n[a];
        info->origin[a] = c->g.o[a];
    }
    info->cell = c->cell;
    info->inv_cell = c->g.inv;
    info->h2 = c->g.h2;
    info->max_neighbors = c->capf;
    info->max_boundary_neighbors = c->capb;
    info->device_bytes = c->dev_bytes;
    return SPH_OK;
}


int sph_read_state(sph_ctx *c, uint32_t mask, const sph_host_view *dst) {
    if (!c || !dst) return SPH_ERR_INVALID;
    c->err.clear();
    const int64_t nf = c->nf, nb = c->nb;
    std::vector<int32_t> id, id_prev;
    std::vector<float4> x4, v4, vin4;
    std::vector<float> f1;
    int rc = d2h(c, id, c->id, nf);
    if (rc) return rc;
    // x, v, rho, K, Kv and the correction are in the current sorted order;
    // the step's other outputs (alpha, kappa, the input velocity, the counts)
    // in the order of the step that wrote them (out_order)
    const sph_ctx::OutOrder oo = c->out_order;
    const int32_t *id_of_out = oo == sph_ctx::OutOrder::Cur ? c->id : oo == sph_ctx::OutOrder::Prev ? c->id2 : c->id_out;
    const uint32_t *ncnt_of_out = oo == sph_ctx::OutOrder::Cur ? c->ncnt
                                  : oo == sph_ctx::OutOrder::Prev ? c->ncnt2 : c->ncnt_out;
    const uint32_t *bcnt_of_out = oo == sph_ctx::OutOrder::Cur ? c->bcnt
                                  : oo == sph_ctx::OutOrder::Prev ? c->bcnt2 : c->bcnt_out;
    if (oo != sph_ctx::OutOrder::Cur && (rc = d2h(c, id_prev, id_of_out, nf))) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const std::vector<int32_t> &idp = oo != sph_ctx::OutOrder::Cur ? id_prev : id;
    auto scatter3 = [&](const std::vector<float4> &src, float *out) {
        for (int64_t s = 0; s < nf; ++s) {
            const int64_t i = id[s];
            out[3 * i] = src[s].x;
            out[3 * i + 1] = src[s].y;
            out[3 * i + 2] = src[s].z;
        }
    };
    auto read1 = [&](const float *d, float *out, const std::vector<int32_t> &ids) -> int {
        int r = d2h(c, f1, d, nf);
        if (r) return r;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t s = 0; s < nf; ++s) out[ids[s]] = f1[s];
        return SPH_OK;
    };
    if ((mask & SPH_FIELD_X) && dst->x) {
        if ((rc = d2h(c, x4, c->x, nf))) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        scatter3(x4, dst->x);
    }
    if ((mask & (SPH_FIELD_V | SPH_FIELD_ACCEL)) && (dst->v || dst->accel)) {
        if ((rc = d2h(c, v4, c->v, nf))) return rc;
        if ((rc = d2h(c, vin4, c->v_in, nf))) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if ((mask & SPH_FIELD_V) && dst->v) scatter3(v4, dst->v);
        if ((mask & SPH_FIELD_ACCEL) && dst->accel) {
            const float idt = c->last_dt > 0 ? 1.0f / c->last_dt : 0.0f;
            std::vector<float4> vin_by_id(std::max<int64_t>(nf, 1));
            for (int64_t s = 0; s < nf; ++s) vin_by_id[idp[s]] = vin4[s];
            for (int64_t s = 0; s < nf; ++s) {
                const int64_t i = id[s];
                dst->accel[3 * i] = (v4[s].x - vin_by_id[i].x) * idt;
                dst->accel[3 * i + 1] = (v4[s].y - vin_by_id[i].y) * idt;
                dst->accel[3 * i + 2] = (v4[s].z - vin_by_id[i].z) * idt;
            }
        }
    }
    if ((mask & SPH_FIELD_DVISC) && dst->dvisc) {
        if (c->dvisc) {
            std::vector<float4> d4;
            if ((rc = d2h(c, d4, c->dvisc, nf))) return rc;
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            scatter3(d4, dst->dvisc);
        } else {
            std::fill(dst->dvisc, dst->dvisc + 3 * nf, 0.0f);
        }
    }
    if ((mask & SPH_FIELD_RHO) && dst->rho && (rc = read1(c->rho, dst->rho, id))) return rc;
    if ((mask & SPH_FIELD_ALPHA) && dst->alpha && (rc = read1(c->alpha, dst->alpha, idp))) return rc;
    if ((mask & SPH_FIELD_K) && dst->K && (rc = read1(c->K, dst->K, id))) return rc;
    if ((mask & SPH_FIELD_KV) && dst->Kv && (rc = read1(c->Kv, dst->Kv, id))) return rc;
    if ((mask & SPH_FIELD_KAPPA) && dst->kappa && (rc = read1(c->kappa_last, dst->kappa, idp))) return rc;
    if ((mask & SPH_FIELD_NBR) && (dst->n_fluid_nbrs || dst->n_boundary_nbrs)) {
        std::vector<uint32_t> a, b;
        if ((rc = d2h(c, a, ncnt_of_out, nf))) return rc;
        if ((rc = d2h(c, b, bcnt_of_out, nf))) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t s = 0; s < nf; ++s) {
            if (dst->n_fluid_nbrs) dst->n_fluid_nbrs[idp[s]] = (int32_t)a[s];
            if (dst->n_boundary_nbrs) dst->n_boundary_nbrs[idp[s]] = (int32_t)b[s];
        }
    }
    if ((mask & (SPH_FIELD_PSI | SPH_FIELD_BOUNDARY)) && (dst->psi || dst->x_boundary || dst->v_boundary)) {
        std::vector<float4> xb4, vb4;
        std::vector<int32_t> bid;
        if ((rc = d2h(c, xb4, c->xb, nb))) return rc;
        if ((rc = d2h(c, vb4, c->vb, nb))) return rc;
        if ((rc = d2h(c, bid, c->bid, nb))) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t s = 0; s < nb; ++s) {
            const int64_t k = bid[s];
            if ((mask & SPH_FIELD_PSI) && dst->psi) dst->psi[k] = xb4[s].w;
            if ((mask & SPH_FIELD_BOUNDARY) && dst->x_boundary) {
                dst->x_boundary[3 * k] = xb4[s].x;
                dst->x_boundary[3 * k + 1] = xb4[s].y;
                dst->x_boundary[3 * k + 2] = xb4[s].z;
            }
            if ((mask & SPH_FIELD_BOUNDARY) && dst->v_boundary) {
                dst->v_boundary[3 * k] = vb4[s].x;
                dst->v_boundary[3 * k + 1] = vb4[s].y;
                dst->v_boundary[3 * k + 2] = vb4[s].z;
            }
        }
    }
    if (mask & SPH_FIELD_RIGID) {
        for (int b = 0; b < c->nr; ++b) {
            if (dst->rigid) dst->rigid[b] = c->rigid[b];
            for (int a = 0; a < 3; ++a) {
                if (dst->rigid_force) dst->rigid_force[3 * b + a] = c->force[3 * b + a];
                if (dst->rigid_torque) dst->rigid_torque[3 * b + a] = c->torque[3 * b + a];
            }
        }
    }
    return SPH_OK;
}

int sph_write_state(sph_ctx *c, uint32_t mask, const sph_host_view *src) {
    if (!c || !src) return SPH_ERR_INVALID;
    c->err.clear();
    c->vmax_ready = false;
    c->build_ahead = false;   // a build queued ahead is stale now: the next step sorts again
    const int64_t nf = c->nf, nb = c->nb;
    std::vector<int32_t> id;
    int rc = d2h(c, id, c->id, nf);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    auto write3 = [&](const float *in, float4 *d, bool keep_w) -> int {
        std::vector<float4> h(std::max<int64_t>(nf, 1));
        if (keep_w) {
            HIP_TRY(c, hipMemcpyAsync(h.data(), d, sizeof(float4) * nf, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
        for (int64_t s = 0; s < nf; ++s) {
            const int64_t i = id[s];
            h[s].x = in[3 * i];
            h[s].y = in[3 * i + 1];
            h[s].z = in[3 * i + 2];
            if (!keep_w) h[s].w = 0.f;
        }
        HIP_TRY(c, hipMemcpyAsync(d, h.data(), sizeof(float4) * nf, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return SPH_OK;
    };
    auto write1 = [&](const float *in, float *d) -> int {
        std::vector<float> h(std::max<int64_t>(nf, 1));
        for (int64_t s = 0; s < nf; ++s) h[s] = in[id[s]];
        HIP_TRY(c, hipMemcpyAsync(d, h.data(), sizeof(float) * nf, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return SPH_OK;
    };
    if ((mask & SPH_FIELD_X) && src->x) {
        if (!finite3(src->x, nf)) return fail(c, SPH_ERR_INVALID, "non-finite position");
        if ((rc = write3(src->x, c->x, false))) return rc;
    }
    if ((mask & SPH_FIELD_V) && src->v && (rc = write3(src->v, c->v, false))) return rc;
    if ((mask & SPH_FIELD_K) && src->K && (rc = write1(src->K, c->K))) return rc;
    if ((mask & SPH_FIELD_KV) && src->Kv && (rc = write1(src->Kv, c->Kv))) return rc;
    if ((mask & SPH_FIELD_RHO) && src->rho) {
        for (int64_t i = 0; i < nf; ++i)
            if (!(src->rho[i] > 0.0f) || !std::isfinite(src->rho[i]))
                return fail(c, SPH_ERR_INVALID, "density must be positive and finite");
        if ((rc = write1(src->rho, c->rho))) return rc;
    }
    if ((mask & SPH_FIELD_DVISC) && src->dvisc) {
        if (!c->dvisc) return fail(c, SPH_ERR_INVALID, "dvisc needs the implicit viscosity model");
        if (!finite3(src->dvisc, nf)) return fail(c, SPH_ERR_INVALID, "non-finite dvisc");
        if ((rc = write3(src->dvisc, c->dvisc, false))) return rc;
    }
    if ((mask & SPH_FIELD_RIGID) && src->rigid) {
        for (int b = 0; b < c->nr; ++b) c->rigid[b] = src->rigid[b];
        if ((rc = upload_poses(c))) return rc;
    }
    if ((mask & SPH_FIELD_BOUNDARY) && (src->x_boundary || src->v_boundary)) {
        std::vector<float4> xb4, vb4;
        std::vector<int32_t> bid;
        if ((rc = d2h(c, xb4, c->xb, nb))) return rc;
        if ((rc = d2h(c, vb4, c->vb, nb))) return rc;
        if ((rc = d2h(c, bid, c->bid, nb))) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t s = 0; s < nb; ++s) {
            const int64_t k = bid[s];
            if (src->x_boundary) {
                xb4[s].x = src->x_boundary[3 * k];
                xb4[s].y = src->x_boundary[3 * k + 1];
                xb4[s].z = src->x_boundary[3 * k + 2];
            }
            if (src->v_boundary) {
                vb4[s].x = src->v_boundary[3 * k];
                vb4[s].y = src->v_boundary[3 * k + 1];
                vb4[s].z = src->v_boundary[3 * k + 2];
                if (vb4[s].x != 0.0f || vb4[s].y != 0.0f || vb4[s].z != 0.0f) c->vb_moving = true;
            }
        }
        HIP_TRY(c, hipMemcpyAsync(c->xb, xb4.data(), sizeof(float4) * nb, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->vb, vb4.data(), sizeof(float4) * nb, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->boundary_dirty = true;
    }
    c->nbr_fresh = false;
    return SPH_OK;
}

int sph_read_neighbors(sph_ctx *c, const sph_nbr_view *d) {
    if (!c || !d) return SPH_ERR_INVALID;
    c->err.clear();
    if (!c->nbr_fresh) return fail(c, SPH_ERR_STATE, "no fresh neighbour lists");
    const int64_t nf = c->nf, nb = c->nb;
    std::vector<uint32_t> key, src, start, cnt, bcnt, lists, bkey, bsrc;
    std::vector<int32_t> id, bid;
    int rc;
    if ((rc = d2h(c, key, c->key, nf)) || (rc = d2h(c, src, c->src, nf)) || (rc = d2h(c, id, c->id, nf)) ||
        (rc = d2h(c, cnt, c->ncnt, nf)) || (rc = d2h(c, bcnt, c->bcnt, nf)) ||
        (rc = d2h(c, bkey, c->bkey, nb)) || (rc = d2h(c, bsrc, c->bsrc, nb)) || (rc = d2h(c, bid, c->bid, nb)))
        return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (d->keys_f)
        for (int64_t s = 0; s < nf; ++s) d->keys_f[s] = key[src[s]];
    if (d->perm_f)
        for (int64_t s = 0; s < nf; ++s) d->perm_f[s] = (uint32_t)id[s];
    if (d->keys_b)
        for (int64_t s = 0; s < nb; ++s) d->keys_b[s] = bkey[bsrc[s]];
    if (d->perm_b)
        for (int64_t s = 0; s < nb; ++s) d->perm_b[s] = (uint32_t)bid[s];
    if (d->start_f)
        HIP_TRY(c, hipMemcpyAsync(d->start_f, c->start_f, sizeof(uint32_t) * (c->ncell + 1), hipMemcpyDeviceToHost, c->stream));
    if (d->start_b)
        HIP_TRY(c, hipMemcpyAsync(d->start_b, c->start_b, sizeof(uint32_t) * (c->ncell + 1), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // lists as sorted indices, CSR by particle
    auto csr = [&](const uint32_t *dev, int32_t cap, const std::vector<uint32_t> &n, uint32_t *counts, uint32_t *out,
                   int64_t outcap) -> int {
        int64_t tot = 0;
        for (int64_t s = 0; s < nf; ++s) tot += std::min<uint32_t>(n[s], (uint32_t)cap);
        if (counts)
            for (int64_t s = 0; s < nf; ++s) counts[s] = n[s];
        if (!out) return SPH_OK;
        if (tot > outcap) return fail(c, SPH_ERR_CAPACITY, "CSR capacity too small");
        // chunks of four entries, chunk-major: entry k of s at 4 ((k/4) nf + s) + k%4
        const int64_t cap4 = ((int64_t)cap + 3) / 4 * 4;
        std::vector<uint32_t> L((size_t)std::max<int64_t>(cap4 * nf, 1));
        HIP_TRY(c, hipMemcpyAsync(L.data(), dev, sizeof(uint32_t) * (size_t)(cap4 * nf), hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        int64_t o = 0;
        for (int64_t q = 0; q < nf; ++q) {
            const uint32_t m = std::min<uint32_t>(n[q], (uint32_t)cap);
            for (uint32_t k = 0; k < m; ++k) out[o++] = L[(size_t)(4 * ((int64_t)(k >> 2) * nf + q) + (k & 3))];
        }
        return SPH_OK;
    };
    if ((rc = csr(c->nlist, c->capf, cnt, d->counts_f, d->lists_f, d->cap_f))) return rc;
    if ((rc = csr(c->blist, c->capb, bcnt, d->counts_b, d->lists_b, d->cap_b))) return rc;
    return SPH_OK;
}

int sph_mlp_create(const float *params, void *hip_stream, sph_mlp **out) {
    g_create_error.clear();
    if (!out || !params) return fail(nullptr, SPH_ERR_INVALID, "params or out is NULL");
    *out = nullptr;
    sph_mlp *m = new (std::nothrow) sph_mlp();
    if (!m) return fail(nullptr, SPH_ERR_OOM, "host allocation failed");
    m->stream = (hipStream_t)hip_stream;
    const int np = sph::mlp_param_count(), nb = sph::mlp_grad_blocks();
    bool ok = hipMalloc(&m->P, sizeof(float) * np) == hipSuccess && hipMalloc(&m->m, sizeof(float) * np) == hipSuccess &&
              hipMalloc(&m->v, sizeof(float) * np) == hipSuccess && hipMalloc(&m->grad, sizeof(float) * np) == hipSuccess &&
              hipMalloc(&m->part, sizeof(float) * (size_t)np * nb) == hipSuccess &&
              hipMalloc(&m->loss_part, sizeof(double) * nb) == hipSuccess &&
              hipMalloc(&m->loss, sizeof(double) * 2) == hipSuccess &&
              hipMalloc(&m->packed, sizeof(uint32_t) * sph::mlp_packed_words()) == hipSuccess;
    if (!ok) {
        sph_mlp_destroy(m);
        return fail(nullptr, SPH_ERR_OOM, "MLP device allocation failed");
    }
    std::vector<float> zero(np, 0.0f);
    ok = hipMemcpyAsync(m->m, zero.data(), sizeof(float) * np, hipMemcpyHostToDevice, m->stream) == hipSuccess &&
         hipMemcpyAsync(m->v, zero.data(), sizeof(float) * np, hipMemcpyHostToDevice, m->stream) == hipSuccess &&
         hipStreamSynchronize(m->stream) == hipSuccess;
    if (!ok || sph_mlp_set_params(m, params) != SPH_OK) {
        sph_mlp_destroy(m);
        return fail(nullptr, SPH_ERR_DEVICE, "MLP upload failed");
    }
    *out = m;
    return SPH_OK;
}

void sph_mlp_destroy(sph_mlp *m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    for (void *p : {(void *)m->P, (void *)m->m, (void *)m->v, (void *)m->grad, (void *)m->part, (void *)m->loss_part,
                    (void *)m->loss, (void *)m->packed})
        if (p) (void)hipFree(p);
    delete m;
}

int sph_mlp_set_params(sph_mlp *m, const float *params) {
    if (!m || !params) return SPH_ERR_INVALID;
    const int np = sph::mlp_param_count();
    m->finite = true;
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(params[i])) m->finite = false;
    if (hipMemcpyAsync(m->P, params, sizeof(float) * np, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
        sph::launch_mlp_pack(m->P, m->packed, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return SPH_ERR_DEVICE;
    return SPH_OK;
}

int sph_mlp_get_params(sph_mlp *m, float *params) {
    if (!m || !params) return SPH_ERR_INVALID;
    if (hipMemcpyAsync(params, m->P, sizeof(float) * sph::mlp_param_count(), hipMemcpyDeviceToHost, m->stream) !=
            hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return SPH_ERR_DEVICE;
    return SPH_OK;
}

int sph_mlp_forward(sph_mlp *m, const float *features, float *y, int64_t n) {
    if (!m || n < 0 || (n > 0 && (!features || !y))) return SPH_ERR_INVALID;
    if (sph::launch_mlp_forward(m->packed, features, n, y, m->stream) != hipSuccess) return SPH_ERR_DEVICE;
    return hipStreamSynchronize(m->stream) == hipSuccess ? SPH_OK : SPH_ERR_DEVICE;
}

namespace {
int mlp_grad_dev(sph_mlp *m, const float *features, const float *targets, int64_t n) {
    if (sph::launch_mlp_grad(m->P, features, targets, n, m->part, m->loss_part, m->grad, m->loss, m->stream) !=
        hipSuccess)
        return SPH_ERR_DEVICE;
    return SPH_OK;
}
}  // namespace

int sph_mlp_grad(sph_mlp *m, const float *features, const float *targets, int64_t n, float *grad, double *loss) {
    if (!m || n <= 0 || !features || !targets) return SPH_ERR_INVALID;
    int rc = mlp_grad_dev(m, features, targets, n);
    if (rc) return rc;
    double l = 0.0;
    if ((grad && hipMemcpyAsync(grad, m->grad, sizeof(float) * sph::mlp_param_count(), hipMemcpyDeviceToHost,
                                m->stream) != hipSuccess) ||
        hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return SPH_ERR_DEVICE;
    if (loss) *loss = l / (double)n;
    return SPH_OK;
}

int sph_mlp_train_step(sph_mlp *m, const float *features, const float *targets, int64_t n, float lr, double *loss) {
    if (!m || n <= 0 || !features || !targets || !(lr > 0)) return SPH_ERR_INVALID;
    int rc = mlp_grad_dev(m, features, targets, n);
    if (rc) return rc;
    m->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, (double)m->step)), c2 = (float)(1.0 - std::pow(b2, (double)m->step));
    if (sph::launch_mlp_adam(m->P, m->grad, m->m, m->v, lr, (float)b1, (float)b2, 1e-8f, c1, c2, m->stream) !=
            hipSuccess ||
        sph::launch_mlp_pack(m->P, m->packed, m->stream) != hipSuccess)
        return SPH_ERR_DEVICE;
    if (loss) {
        double l = 0.0;
        if (hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
            hipStreamSynchronize(m->stream) != hipSuccess)
            return SPH_ERR_DEVICE;
        *loss = l / (double)n;
    }
    return SPH_OK;
}

int sph_set_warm_start(sph_ctx *c, int32_t mode, sph_mlp *mlp) {
    if (!c || mode < SPH_WARM_ZERO || mode > SPH_WARM_LEARNED) return SPH_ERR_INVALID;
    c->warm_fallback = false;
    if (mode == SPH_WARM_LEARNED) {
        if (!mlp) return fail(c, SPH_ERR_INVALID, "learned warm start needs an MLP");
        if (c->P.solver != SPH_SOLVER_DFSPH)
            return fail(c, SPH_ERR_INVALID, "the learned warm start needs the DFSPH solver");
        if (!mlp->finite) {
            c->warm_fallback = true;
            c->warm_mode = SPH_WARM_PREVIOUS;
            c->mlp = nullptr;
            return SPH_OK;
        }
        c->mlp = mlp;
    } else {
        c->mlp = nullptr;
    }
    c->warm_mode = mode;
    return SPH_OK;
}

int sph_enable_trace(sph_ctx *c, float *features, float *targets, int64_t capacity) {
    if (!c || capacity < 0 || (features && !targets)) return SPH_ERR_INVALID;
    c->trace_feat = features;
    c->trace_target = targets;
    c->trace_cap = features ? capacity : 0;
    c->trace_rows = 0;
    return SPH_OK;
}

int sph_trace_rows(const sph_ctx *c, int64_t *rows) {
    if (!c || !rows) return SPH_ERR_INVALID;
    *rows = c->trace_rows;
    return SPH_OK;
}

int sph_set_forced_iters(sph_ctx *c, int32_t div, int32_t dens) {
    if (!c) return SPH_ERR_INVALID;
    c->forced_div = div;
    c->forced_dens = dens;
    return SPH_OK;
}

int sph_profile_enable(sph_ctx *c, int32_t enable) {
    if (!c) return SPH_ERR_INVALID;
    prof_resolve(c);
    c->prof = enable != 0;
    if (enable) c->prof_total.clear();
    return SPH_OK;
}

int sph_profile_only(sph_ctx *c, const char *kernel) {
    if (!c) return SPH_ERR_INVALID;
    c->prof_only = kernel ? kernel : "";
    return SPH_OK;
}

int sph_profile_read(sph_ctx *c, const char *kernel, int64_t *launches, double *total_ms, double *bytes) {
    if (!c || !kernel) return SPH_ERR_INVALID;
    prof_resolve(c);
    auto it = c->prof_total.find(kernel);
    const ProfTotal t = it == c->prof_total.end() ? ProfTotal{} : it->second;
    if (launches) *launches = t.launches;
    if (total_ms) *total_ms = t.ms;
    if (bytes) *bytes = t.bytes;
    return SPH_OK;
}

}  // extern "C"
