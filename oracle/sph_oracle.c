/*
 * sph_oracle.c -- plain, slow FP64 CPU oracle for one DFSPH time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load or call
 * this library; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the HIP library.
 *
 * Every function follows the paper (arXiv 2403.11156, "Journey into SPH
 * Simulation") and the readings listed with it:
 *   - density summation, Eq. (4); Akinci boundary density, Eq. (12);
 *   - Akinci boundary mass Psi, Eq. (11);
 *   - pressure acceleration, Eq. (7), with the boundary term of Eq. (13) and
 *     its reaction on the rigid body, Eq. (14);
 *   - the velocity-source (Eq. 10) and density-source (Eqs. 8-9) pressure
 *     solves, iterated as in Algorithm 2 (DFSPH, which uses both);
 *   - the step skeleton of Algorithm 1 (non-pressure, pressure, symplectic
 *     Euler);
 *   - explicit viscosity Eq. (15), implicit viscosity Eqs. (16)-(19) solved by
 *     matrix-free conjugate gradients (Sec. 4.2);
 *   - the uniform grid with prefix sums (Sec. 5.6) for the neighbour search;
 *   - the rigid bodies the paper leaves to a physics engine (Sec. 4.2):
 *     Newton-Euler in FP64, the weak coupling of Sec. 3.5, the interlinked
 *     (strong) coupling that Sec. 6 names as future work, and frictionless
 *     contact of the bodies' sample points; these are our own models, each
 *     pinned by closed forms and conservation laws in the tests (a body at
 *     rest takes its weight, head-on boxes stop one spacing apart, impulse
 *     pairs keep momentum and angular momentum, a body a trillion times
 *     heavier reproduces the weak coupling).
 *
 * Neighbour membership and cell keys are decided in FP32 (the state is FP32)
 * exactly as the readings fix them; everything else is FP64 from the FP32
 * inputs widened exactly.  Alongside each field the oracle carries a running
 * error scale S (the same formula with every operand replaced by its absolute
 * value or scale and every a-b by |a|+|b|; the componentwise forward-error
 * bound of Higham, "Accuracy and Stability of Numerical Algorithms", ch. 3).
 * A difference of two exact FP32 inputs (x_i - x_j) is one rounding of its
 * result, so its scale is its own magnitude.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so the
 * FP32 key and distance arithmetic is the plain IEEE sequence).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Parameters and I/O records (mirrored by the Python wrapper).              */
/* ------------------------------------------------------------------------ */
typedef struct or_params {
    double r, h, rho0;
    double gravity[3];
    double domain_min[3], domain_max[3];
    double eta_density, eta_divergence;
    int32_t max_iters;
    double dt_max, cfl_lambda;
    int32_t visc_model; /* 0 none, 1 XSPH, 2 Eq. 15, 3 implicit Eqs. 16-19 */
    double visc;        /* XSPH epsilon, or kinematic viscosity nu [m^2/s] */
    double cg_tol;
    int32_t cg_max_iters;
    int32_t warm_start; /* 0 zero, 1 previous, 2 learned */
    int32_t forced_div, forced_dens; /* >= 0: run exactly that many iterations */
    int32_t n_rigid;
    double warm_factor;   /* PREVIOUS warm start: K0 = warm_factor * K_prev */
    int32_t solver;       /* 0 DFSPH, 1 WCSPH (equation of state, one pressure pass),
                             2 PCISPH (density solve with the prototype stiffness factor) */
    double wcsph_k, wcsph_gamma;  /* WCSPH stiffness [Pa] and exponent */
    double cg_warm_factor;        /* implicit-viscosity CG start: x0 = b + cg_warm_factor dvisc_prev */
    double alpha_max_factor;      /* DFSPH factor capped at alpha_max_factor * alpha_ref (0: no cap) */
    double eta_density_max;       /* > 0: the density solve also bounds the largest compression */
    int32_t rigid_coupling;       /* 0 weak (bodies move after the fluid solve), 1 strong (every
                                     pressure pass moves them: the interlinked coupling of
                                     Sec. 6's outlook, in our reading) */
    int32_t rigid_contact;        /* 0 a stand-in that keeps bodies inside the tank, 1 rigid
                                     contact between bodies and with the tank (our model) */
} or_params;

typedef struct or_rigid {
    double mass, inertia[3], com[3], quat[4], vel[3], omega[3];
} or_rigid;

/* learned warm start: out[i] = MLP(features[i*5 .. i*5+4]) and out[n + i] the
 * error scale of that prediction (in the units of the S fields) given the
 * features' error scales S_features[i*5 ..] */
typedef void (*or_mlp_fn)(const double *features, const double *S_features, int64_t n, double *out, void *user);

typedef struct or_in {
    int64_t nf, nb;
    const float *xf, *vf;      /* [nf][3] */
    const float *K, *Kv;       /* [nf] previous accumulated stiffness */
    const float *xb, *vb;      /* [nb][3] */
    const int32_t *body;       /* [nb], -1 static */
    const double *local;       /* [nb][3] body-frame offsets (rigid only) */
    const or_rigid *rigid;     /* [n_rigid] state at step start */
    or_mlp_fn mlp;
    void *mlp_user;
    int32_t brute_force;       /* 1: O(N^2) neighbour sets, 0: oracle grid */
    const float *dvisc;        /* [nf][3] previous implicit-viscosity correction v* - b (NULL: zero) */
    const float *rho_prev;     /* [nf] previous step's density (NULL: rho0), for the divergence warm start */
} or_in;

typedef struct or_out {
    /* fields, original (id) order */
    double *x, *v, *rho, *alpha, *K, *Kv, *kappa, *accel, *psi; /* psi: [nb] */
    double *S_x, *S_v, *S_K, *S_Kv, *S_kappa, *S_accel, *S_alpha;
    int32_t *nf_count, *nb_count;
    double *features;          /* [nf][5] learned-warm-start inputs (may be NULL) */
    double *target;            /* [nf] learned-warm-start target (may be NULL) */
    double *S_features, *S_target; /* their error scales (with features/target) */
    float *xb_new, *vb_new;    /* [nb][3] boundary state for the next step */
    or_rigid *rigid_new;       /* [n_rigid] */
    double *force, *torque;    /* [n_rigid][3] */
    double *S_force, *S_torque;/* [n_rigid][3] error scales */
    /* stats */
    double dt;
    int32_t iters_div, iters_dens, converged_div, converged_dens, cg_iters;
    double err_div, err_dens, S_err_div, S_err_dens, cg_resid;
    double err_div_hist[128], err_dens_hist[128];
    double *dvisc;             /* [nf][3] this step's implicit-viscosity correction v* - b (may be NULL) */
    double err_dens_max;       /* largest predicted compression / rho0 after the density solve */
    double err_dens_max_hist[128];
} or_out;

/* ------------------------------------------------------------------------ */
/* Cubic spline kernel with support radius h (reading of Sec. 3.2; the paper  */
/* leaves W open, the form is the one of its SPH tutorial reference).        */
/*   W = k f(q), q = r/h, k = 8/(pi h^3)                                      */
/*   f = 6(q^3 - q^2) + 1 (q <= 1/2), 2(1-q)^3 (1/2 < q <= 1), 0 otherwise    */
/* ------------------------------------------------------------------------ */
double or_kernel_k(double h) { return 8.0 / (M_PI * h * h * h); }

double or_W(double r, double h) {
    double q = r / h, k = or_kernel_k(h);
    if (q <= 0.5) return k * (6.0 * (q * q * q - q * q) + 1.0);
    if (q <= 1.0) { double t = 1.0 - q; return k * 2.0 * t * t * t; }
    return 0.0;
}

/* |W| scale: the same polynomial with absolute values */
static double W_scale(double r, double h) {
    double q = r / h, k = or_kernel_k(h);
    if (q <= 0.5) return k * (6.0 * (q * q * q + q * q) + 1.0);
    if (q <= 1.0) { double t = 1.0 + q; return k * 2.0 * t * t * t; }
    return 0.0;
}

/* dW/dr */
double or_dWdr(double r, double h) {
    double q = r / h, k = or_kernel_k(h);
    if (q <= 0.5) return k / h * 6.0 * (3.0 * q * q - 2.0 * q);
    if (q <= 1.0) { double t = 1.0 - q; return -k / h * 6.0 * t * t; }
    return 0.0;
}

static double dWdr_scale(double r, double h) {
    double q = r / h, k = or_kernel_k(h);
    if (q <= 0.5) return k / h * 6.0 * (3.0 * q * q + 2.0 * q);
    if (q <= 1.0) { double t = 1.0 + q; return k / h * 6.0 * t * t; }
    return 0.0;
}

/* grad_i W(x_i - x_j): dW/dr * x_ij / |x_ij|; zero for coincident points */
void or_gradW(const double xij[3], double h, double g[3]) {
    double r = sqrt(xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2]);
    if (r <= 0.0) { g[0] = g[1] = g[2] = 0.0; return; }
    double f = or_dWdr(r, h) / r;
    g[0] = f * xij[0]; g[1] = f * xij[1]; g[2] = f * xij[2];
}

static void gradW_scale(const double xij[3], double h, double sg[3]) {
    double r = sqrt(xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2]);
    if (r <= 0.0) { sg[0] = sg[1] = sg[2] = 0.0; return; }
    double f = dWdr_scale(r, h) / r;
    sg[0] = f * fabs(xij[0]); sg[1] = f * fabs(xij[1]); sg[2] = f * fabs(xij[2]);
}

/* ------------------------------------------------------------------------ */
/* Uniform grid (the "prefix sum" grid of Sec. 5.6; cell reading: cell edge  */
/* fl32(h(1+2^-10)), reciprocal fl32(1/cell), origin fl32(min - cell),       */
/* n_a = ceil((max-min)/cell) + 2 cells per axis, keys clamped, x fastest).  */
/* ------------------------------------------------------------------------ */
typedef struct or_grid {
    float cell, inv, o[3], h2;
    int32_t n[3];
} or_grid;

void or_grid_make(double h, const double dmin[3], const double dmax[3], or_grid *g) {
    g->cell = (float)(h * (1.0 + 1.0 / 1024.0));
    g->inv = 1.0f / g->cell;
    for (int a = 0; a < 3; ++a) {
        g->o[a] = (float)(dmin[a] - (double)g->cell);
        g->n[a] = (int32_t)ceil((dmax[a] - dmin[a]) / (double)g->cell) + 2;
    }
    float hf = (float)h;
    g->h2 = hf * hf;
}

static int32_t cell_coord(float x, float o, float inv, int32_t n) {
    float t = (x - o) * inv;          /* two FP32 roundings, no FMA */
    float f = floorf(t);
    if (!(f >= 0.0f)) return 0;        /* also catches NaN */
    if (f > (float)(n - 1)) return n - 1;
    return (int32_t)f;
}

uint32_t or_cell_key(const or_grid *g, const float x[3]) {
    int32_t cx = cell_coord(x[0], g->o[0], g->inv, g->n[0]);
    int32_t cy = cell_coord(x[1], g->o[1], g->inv, g->n[1]);
    int32_t cz = cell_coord(x[2], g->o[2], g->inv, g->n[2]);
    return (uint32_t)(cx + g->n[0] * (cy + g->n[1] * cz));
}

void or_cell_keys(const or_grid *g, const float *x, int64_t n, uint32_t *key) {
    for (int64_t i = 0; i < n; ++i) key[i] = or_cell_key(g, x + 3 * i);
}

/* order by (key, id); the id is the array index */
static const uint32_t *g_sort_keys;
static int cmp_key_id(const void *a, const void *b) {
    uint32_t ia = *(const uint32_t *)a, ib = *(const uint32_t *)b;
    uint32_t ka = g_sort_keys[ia], kb = g_sort_keys[ib];
    if (ka != kb) return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

/* perm[s] = id of the particle at sorted position s */
void or_sort_perm(const uint32_t *key, int64_t n, uint32_t *perm) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    g_sort_keys = key;
    qsort(perm, (size_t)n, sizeof(uint32_t), cmp_key_id);
}

/* start[c] = first sorted position with key >= c; start[ncell] = n */
void or_cell_start(const uint32_t *key, const uint32_t *perm, int64_t n, int64_t ncell, uint32_t *start) {
    int64_t s = 0;
    for (int64_t c = 0; c <= ncell; ++c) {
        while (s < n && key[perm[s]] < (uint32_t)c) ++s;
        start[c] = (uint32_t)s;
    }
}

/* FP32 squared distance ((dx*dx + dy*dy) + dz*dz), no FMA */
static float dist2_f32(const float *a, const float *b) {
    float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

/*
 * Brute-force neighbour sets in sorted-index space: for each query q (in
 * sorted order) all candidates c (ascending sorted index) with d^2 < h^2;
 * with same_set, c == q is excluded.  Output is CSR (counts + concatenated
 * lists).  Returns the total, or -1 if out_cap is too small.
 */
int64_t or_neighbors_brute(const float *xq, int64_t nq, const float *xc, int64_t nc, float h2,
                           int32_t same_set, uint32_t *counts, uint32_t *out, int64_t out_cap) {
    int64_t tot = 0;
    for (int64_t i = 0; i < nq; ++i) {
        uint32_t cnt = 0;
        for (int64_t j = 0; j < nc; ++j) {
            if (same_set && j == i) continue;
            if (dist2_f32(xq + 3 * i, xc + 3 * j) < h2) {
                if (tot >= out_cap) return -1;
                out[tot++] = (uint32_t)j;
                ++cnt;
            }
        }
        counts[i] = cnt;
    }
    return tot;
}

/*
 * The oracle's own grid search: the 27-cell stencil walked dz, dy outer and
 * the contiguous cx-1..cx+1 run inner, which yields ascending sorted indices.
 * xq/xc are in their sorted orders; start is the candidate set's cell table.
 */
/* the neighbours of one query in stencil order; writes them to out (if not
 * NULL) and returns their number */
static uint32_t grid_query(const or_grid *g, const float *xi, int64_t i, const float *xc, const uint32_t *start,
                           int32_t same_set, uint32_t *out) {
    int32_t cx = cell_coord(xi[0], g->o[0], g->inv, g->n[0]);
    int32_t cy = cell_coord(xi[1], g->o[1], g->inv, g->n[1]);
    int32_t cz = cell_coord(xi[2], g->o[2], g->inv, g->n[2]);
    uint32_t cnt = 0;
    for (int32_t dz = -1; dz <= 1; ++dz) {
        int32_t z = cz + dz;
        if (z < 0 || z >= g->n[2]) continue;
        for (int32_t dy = -1; dy <= 1; ++dy) {
            int32_t y = cy + dy;
            if (y < 0 || y >= g->n[1]) continue;
            int32_t x0 = cx > 0 ? cx - 1 : 0;
            int32_t x1 = cx < g->n[0] - 1 ? cx + 1 : g->n[0] - 1;
            int64_t row = (int64_t)g->n[0] * (y + (int64_t)g->n[1] * z);
            uint32_t b = start[row + x0], e = start[row + x1 + 1];
            for (uint32_t j = b; j < e; ++j) {
                if (same_set && (int64_t)j == i) continue;
                if (dist2_f32(xi, xc + 3 * (int64_t)j) < g->h2) {
                    if (out) out[cnt] = j;
                    ++cnt;
                }
            }
        }
    }
    return cnt;
}

/* counts first, then each query's list at its offset (independent queries) */
int64_t or_neighbors_grid(const or_grid *g, const float *xq, int64_t nq, const float *xc,
                          const uint32_t *start, int32_t same_set, uint32_t *counts, uint32_t *out,
                          int64_t out_cap) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nq; ++i) counts[i] = grid_query(g, xq + 3 * i, i, xc, start, same_set, NULL);
    int64_t tot = 0;
    for (int64_t i = 0; i < nq; ++i) tot += counts[i];
    if (tot > out_cap) return -1;
    int64_t *off = malloc(sizeof(int64_t) * (nq + 1));
    off[0] = 0;
    for (int64_t i = 0; i < nq; ++i) off[i + 1] = off[i] + counts[i];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nq; ++i) grid_query(g, xq + 3 * i, i, xc, start, same_set, out + off[i]);
    free(off);
    return tot;
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets in id space (CSR), built from the sorted-order search.     */
/* ------------------------------------------------------------------------ */
typedef struct csr {
    int64_t *start; /* [n+1] */
    uint32_t *idx;
} csr;

static void csr_free(csr *c) { free(c->start); free(c->idx); c->start = NULL; c->idx = NULL; }

/* sort a point set, returns sorted xs and perm */
static void sort_points(const or_grid *g, const float *x, int64_t n, uint32_t **perm_out, float **xs_out,
                        uint32_t **start_out) {
    int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
    uint32_t *key = malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *perm = malloc(sizeof(uint32_t) * (n ? n : 1));
    float *xs = malloc(sizeof(float) * 3 * (n ? n : 1));
    uint32_t *start = malloc(sizeof(uint32_t) * (ncell + 1));
    or_cell_keys(g, x, n, key);
    or_sort_perm(key, n, perm);
    for (int64_t s = 0; s < n; ++s) memcpy(xs + 3 * s, x + 3 * (int64_t)perm[s], 3 * sizeof(float));
    or_cell_start(key, perm, n, ncell, start);
    free(key);
    *perm_out = perm; *xs_out = xs; *start_out = start;
}

/*
 * Neighbour CSR in id space for queries q (ids) against candidates c (ids).
 * Lists keep the ascending sorted-index order of the candidate set.
 */
static int build_csr(const or_grid *g, const float *xq_sorted, const uint32_t *perm_q, int64_t nq,
                     const float *xc_sorted, const uint32_t *perm_c, const uint32_t *start_c, int64_t nc,
                     int32_t same_set, int32_t brute, csr *out) {
    int64_t cap = 64 * (nq + 1);
    uint32_t *counts = malloc(sizeof(uint32_t) * (nq ? nq : 1));
    uint32_t *lst = NULL;
    int64_t tot;
    for (;;) {
        lst = malloc(sizeof(uint32_t) * cap);
        if (brute)
            tot = or_neighbors_brute(xq_sorted, nq, xc_sorted, nc, g->h2, same_set, counts, lst, cap);
        else
            tot = or_neighbors_grid(g, xq_sorted, nq, xc_sorted, start_c, same_set, counts, lst, cap);
        if (tot >= 0) break;
        free(lst);
        cap *= 2;
    }
    /* sorted-space CSR -> id-space CSR */
    int64_t *soff = malloc(sizeof(int64_t) * (nq + 1));
    soff[0] = 0;
    for (int64_t s = 0; s < nq; ++s) soff[s + 1] = soff[s] + counts[s];
    out->start = malloc(sizeof(int64_t) * (nq + 1));
    out->idx = malloc(sizeof(uint32_t) * (tot ? tot : 1));
    int64_t *cnt_id = calloc((size_t)(nq + 1), sizeof(int64_t));
    for (int64_t s = 0; s < nq; ++s) cnt_id[perm_q[s]] = counts[s];
    out->start[0] = 0;
    for (int64_t i = 0; i < nq; ++i) out->start[i + 1] = out->start[i] + cnt_id[i];
    for (int64_t s = 0; s < nq; ++s) {
        int64_t id = perm_q[s];
        for (int64_t k = 0; k < (int64_t)counts[s]; ++k)
            out->idx[out->start[id] + k] = perm_c[lst[soff[s] + k]];
    }
    free(cnt_id); free(soff); free(lst); free(counts);
    (void)nc;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static void quat_to_R(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void cross(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* body-frame offsets r_k = R(q)^T (x_k - c) for the rigid particles */
void or_rigid_local(const float *xb, const int32_t *body, int64_t nb, const or_rigid *rigid, double *local) {
    for (int64_t k = 0; k < nb; ++k) {
        local[3 * k] = local[3 * k + 1] = local[3 * k + 2] = 0.0;
        if (body[k] < 0) continue;
        const or_rigid *b = &rigid[body[k]];
        double R[9], d[3];
        quat_to_R(b->quat, R);
        for (int a = 0; a < 3; ++a) d[a] = (double)xb[3 * k + a] - b->com[a];
        for (int a = 0; a < 3; ++a) local[3 * k + a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Akinci boundary mass, Eq. (11): Psi_b = rho0 / sum_k W_bk over the        */
/* boundary neighbours of b, self included (every body and the tank).        */
/* ------------------------------------------------------------------------ */
static void boundary_psi(const or_params *p, const double *xb, int64_t nb, const csr *bb, double *psi) {
    double k0 = or_W(0.0, p->h);
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        double s = k0;
        for (int64_t e = bb->start[b]; e < bb->start[b + 1]; ++e) {
            int64_t c = bb->idx[e];
            double d[3] = {xb[3 * b] - xb[3 * c], xb[3 * b + 1] - xb[3 * c + 1], xb[3 * b + 2] - xb[3 * c + 2]};
            s += or_W(sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), p->h);
        }
        psi[b] = p->rho0 / s;
    }
}

/* public wrapper: Psi for an FP32 boundary set (brute-force neighbours) */
void or_boundary_psi(const or_params *p, const float *xb32, int64_t nb, double *psi) {
    or_grid g;
    or_grid_make(p->h, p->domain_min, p->domain_max, &g);
    uint32_t *perm, *start;
    float *xs;
    sort_points(&g, xb32, nb, &perm, &xs, &start);
    csr bb;
    build_csr(&g, xs, perm, nb, xs, perm, start, nb, 1, nb <= 20000, &bb);
    double *xb = malloc(sizeof(double) * 3 * (nb ? nb : 1));
    for (int64_t i = 0; i < 3 * nb; ++i) xb[i] = xb32[i];
    boundary_psi(p, xb, nb, &bb, psi);
    free(xb); csr_free(&bb); free(perm); free(xs); free(start);
}

/* ------------------------------------------------------------------------ */
/* The step                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct world {
    const or_params *p;
    int64_t nf, nb;
    double m, h, k0, dt;
    double *x, *v, *Sv;            /* fluid [nf][3] */
    double *xb, *vb, *psi;         /* boundary */
    csr ff, fb;
    double *rho, *alpha, *Salpha;
    /* strong coupling: the bodies' velocities during the step, their world
     * inverse inertia, and the reactions summed over the step's passes */
    int32_t nr, strong;
    const int32_t *body;           /* [nb] body of each boundary particle, -1 static */
    const float *xb32;             /* [nb][3] boundary positions as stored (FP32) */
    or_rigid *bs;                  /* [nr] state during the step */
    double *Iwinv, *Iw;            /* [nr][9] */
    double *F, *T, *SF, *ST;       /* [nr][3] */
} world;

#define FOR_F(i, e) for (int64_t e = w->ff.start[i]; e < w->ff.start[(i) + 1]; ++e)
#define FOR_B(i, e) for (int64_t e = w->fb.start[i]; e < w->fb.start[(i) + 1]; ++e)

static void xij_f(const world *w, int64_t i, int64_t j, double d[3]) {
    for (int a = 0; a < 3; ++a) d[a] = w->x[3 * i + a] - w->x[3 * j + a];
}
static void xij_b(const world *w, int64_t i, int64_t k, double d[3]) {
    for (int a = 0; a < 3; ++a) d[a] = w->x[3 * i + a] - w->xb[3 * k + a];
}

/* Eq. (12) density, and the DFSPH factor alpha (reading: alpha = rho / D,
 * D = |sum_F m gradW + sum_B Psi gradW|^2 + sum_F |m gradW|^2, alpha = 0 when
 * D <= 1e-12 of a bulk particle's D (no neighbour gradient), and alpha capped
 * at alpha_max_factor times
 * the bulk-lattice factor alpha_ref = 2.35376 (2r)^2 / rho0: a particle that
 * sees a few neighbours at the edge of the support has a vanishing gradient
 * and an unbounded factor, and the stiffness it accumulates would be carried
 * into the next step, where the same pair may sit much closer). */
static double alpha_cap(const or_params *p) {
    const double s = 2.0 * p->r;
    return p->alpha_max_factor > 0.0 ? p->alpha_max_factor * 2.35376 * s * s / p->rho0 : 0.0;
}

/* D of a bulk lattice point: sum over its neighbours (spacing 2r, inside the
 * support) of |m gradW|^2 (the gradient sum itself vanishes by symmetry) */
static double bulk_D(const or_params *p) {
    const double s = 2.0 * p->r, h = p->h, m = p->rho0 * s * s * s;
    const int n = (int)ceil(h / s);
    double sum = 0.0;
    for (int a = -n; a <= n; ++a)
        for (int b = -n; b <= n; ++b)
            for (int c = -n; c <= n; ++c) {
                const double d = s * sqrt((double)(a * a + b * b + c * c));
                if (d == 0.0 || d >= h) continue;
                const double g = m * or_dWdr(d, h);
                sum += g * g;
            }
    return sum;
}

static void density_alpha(world *w) {
    const double m = w->m, h = w->h;
    const double amax = alpha_cap(w->p);
    /* no factor below 1e-12 of the bulk D: a neighbour sitting within
     * rounding of the support's edge gives a vanishing gradient, zero in
     * FP32 where FP64 still sees ~1e-30 of the bulk, so both precisions
     * decide alike (the bulk is ~1e9 in SI units) */
    const double Dmin = 1e-12 * bulk_D(w->p);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < w->nf; ++i) {
        double rho = m * w->k0, g[3] = {0, 0, 0}, Sg[3] = {0, 0, 0}, sq = 0.0;
        FOR_F(i, e) {
            int64_t j = w->ff.idx[e];
            double d[3], gw[3], sg[3];
            xij_f(w, i, j, d);
            rho += m * or_W(sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), h);
            or_gradW(d, h, gw);
            gradW_scale(d, h, sg);
            for (int a = 0; a < 3; ++a) { g[a] += m * gw[a]; Sg[a] += m * sg[a]; }
            sq += m * m * (gw[0] * gw[0] + gw[1] * gw[1] + gw[2] * gw[2]);
        }
        FOR_B(i, e) {
            int64_t k = w->fb.idx[e];
            double d[3], gw[3], sg[3];
            xij_b(w, i, k, d);
            rho += w->psi[k] * or_W(sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), h);
            or_gradW(d, h, gw);
            gradW_scale(d, h, sg);
            for (int a = 0; a < 3; ++a) { g[a] += w->psi[k] * gw[a]; Sg[a] += w->psi[k] * sg[a]; }
        }
        double D = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + sq;
        double SD = Sg[0] * Sg[0] + Sg[1] * Sg[1] + Sg[2] * Sg[2] + sq;
        w->rho[i] = rho;
        if (D > Dmin) {
            /* the cap is 1-Lipschitz, so the uncapped scale still bounds the error */
            w->alpha[i] = rho / D;
            w->Salpha[i] = rho / D + rho * SD / (D * D);
            if (amax > 0.0 && w->alpha[i] > amax) w->alpha[i] = amax;
        } else {
            w->alpha[i] = 0.0;
            w->Salpha[i] = 0.0;
        }
    }
}

/*
 * Rate of density change (reading of Eq. 6 and Eq. 9 in the DFSPH form):
 *   d_i = sum_F m (v_i - v_j).gradW_ij + sum_B Psi_k (v_i - v_k).gradW_ik
 */
static void divergence(const world *w, const double *v, const double *Sv, double *d, double *Sd) {
    const double m = w->m, h = w->h;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < w->nf; ++i) {
        double s = 0.0, S = 0.0;
        FOR_F(i, e) {
            int64_t j = w->ff.idx[e];
            double x[3], gw[3], sg[3];
            xij_f(w, i, j, x);
            or_gradW(x, h, gw);
            gradW_scale(x, h, sg);
            for (int a = 0; a < 3; ++a) {
                s += m * (v[3 * i + a] - v[3 * j + a]) * gw[a];
                S += m * (Sv[3 * i + a] + Sv[3 * j + a]) * sg[a];
            }
        }
        FOR_B(i, e) {
            int64_t k = w->fb.idx[e];
            double x[3], gw[3], sg[3];
            xij_b(w, i, k, x);
            or_gradW(x, h, gw);
            gradW_scale(x, h, sg);
            for (int a = 0; a < 3; ++a) {
                s += w->psi[k] * (v[3 * i + a] - w->vb[3 * k + a]) * gw[a];
                S += w->psi[k] * (Sv[3 * i + a] + fabs(w->vb[3 * k + a])) * sg[a];
            }
        }
        d[i] = s;
        Sd[i] = S;
    }
}

/*
 * Pressure velocity update (Eq. 7 with p_i/rho_i^2 = kappa_i/rho_i, and the
 * boundary term of Eq. 13 using the fluid particle's own pressure):
 *   v_i -= dt [ sum_F m (kr_i + kr_j) gradW_ij + sum_B Psi_k kr_i gradW_ik ],
 * kr = kappa / rho.  impulse (optional, [n_rigid][6]) collects the Eq. 14
 * reaction on the bodies (force and torque about the body centre).
 */
/* pressure velocity update with kappa_j / den_j in place of kappa_j / rho_j */
static void pressure_update_den(const world *w, const double *kappa, const double *Skappa, const double *den,
                                double *v, double *Sv) {
    const double m = w->m, h = w->h, dt = w->dt;
    double *dv = malloc(sizeof(double) * 3 * (w->nf ? w->nf : 1));
    double *Sdv = malloc(sizeof(double) * 3 * (w->nf ? w->nf : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < w->nf; ++i) {
        double kri = kappa[i] / den[i], Skri = (Skappa[i] + fabs(kappa[i])) / den[i];
        double acc[3] = {0, 0, 0}, Sacc[3] = {0, 0, 0};
        FOR_F(i, e) {
            int64_t j = w->ff.idx[e];
            double krj = kappa[j] / den[j], Skrj = (Skappa[j] + fabs(kappa[j])) / den[j];
            double x[3], gw[3], sg[3];
            xij_f(w, i, j, x);
            or_gradW(x, h, gw);
            gradW_scale(x, h, sg);
            for (int a = 0; a < 3; ++a) {
                acc[a] += m * (kri + krj) * gw[a];
                Sacc[a] += m * (Skri + Skrj) * sg[a];
            }
        }
        FOR_B(i, e) {
            int64_t k = w->fb.idx[e];
            double x[3], gw[3], sg[3];
            xij_b(w, i, k, x);
            or_gradW(x, h, gw);
            gradW_scale(x, h, sg);
            for (int a = 0; a < 3; ++a) {
                acc[a] += w->psi[k] * kri * gw[a];
                Sacc[a] += w->psi[k] * Skri * sg[a];
            }
        }
        for (int a = 0; a < 3; ++a) { dv[3 * i + a] = dt * acc[a]; Sdv[3 * i + a] = dt * Sacc[a]; }
    }
    for (int64_t i = 0; i < 3 * w->nf; ++i) { v[i] -= dv[i]; Sv[i] += Sdv[i]; }
    free(dv); free(Sdv);
}

/* Boundary velocities of the bodies' particles from the bodies' state:
 * v_k = fl32(V + w x (x_k - c)) with x_k the stored FP32 position. */
static void body_boundary_velocities(world *w) {
    for (int64_t k = 0; k < w->nb; ++k) {
        const int32_t b = w->body[k];
        if (b < 0) continue;
        const or_rigid *s = &w->bs[b];
        double r[3], wx[3];
        for (int a = 0; a < 3; ++a) r[a] = (double)w->xb32[3 * k + a] - s->com[a];
        wx[0] = s->omega[1] * r[2] - s->omega[2] * r[1];
        wx[1] = s->omega[2] * r[0] - s->omega[0] * r[2];
        wx[2] = s->omega[0] * r[1] - s->omega[1] * r[0];
        for (int a = 0; a < 3; ++a) w->vb[3 * k + a] = (double)(float)(s->vel[a] + wx[a]);
    }
}

/* Strong coupling (our reading of the interlinked coupling that Sec. 6 names
 * as future work): the reaction of one pressure pass on each
 * body, Eq. (14) with the pass's stiffness over density,
 *   F_b = sum_i sum_{k in b} m Psi_k (kappa_i / den_i) gradW_ik,
 *   tau_b = sum (x_k - c_b) x F_ik,
 * applied to the body at once (V += dt F/M, w += dt I_w^-1 tau), summed into
 * the step's reaction, and the body's boundary velocities refreshed for the
 * next pass. */
static void couple_pass(world *w, const double *kappa, const double *Skappa, const double *den) {
    if (!w->strong || w->nr == 0) return;
    double *F = calloc((size_t)(6 * w->nr), sizeof(double)), *SF = calloc((size_t)(6 * w->nr), sizeof(double));
    for (int64_t i = 0; i < w->nf; ++i) {
        FOR_B(i, e) {
            const int64_t k = w->fb.idx[e];
            const int32_t b = w->body[k];
            if (b < 0) continue;
            double x[3], gw[3], sg[3], f[3], r[3], t[3];
            xij_b(w, i, k, x);
            or_gradW(x, w->h, gw);
            gradW_scale(x, w->h, sg);
            const double c = w->m * w->psi[k] * kappa[i] / den[i];
            const double Sc = w->m * w->psi[k] * (Skappa[i] + fabs(kappa[i])) / den[i];
            for (int a = 0; a < 3; ++a) {
                f[a] = c * gw[a];
                r[a] = w->xb[3 * k + a] - w->bs[b].com[a];
            }
            t[0] = r[1] * f[2] - r[2] * f[1];
            t[1] = r[2] * f[0] - r[0] * f[2];
            t[2] = r[0] * f[1] - r[1] * f[0];
            for (int a = 0; a < 3; ++a) {
                F[6 * b + a] += f[a];
                F[6 * b + 3 + a] += t[a];
                SF[6 * b + a] += Sc * sg[a];
            }
            SF[6 * b + 3] += fabs(r[1]) * Sc * sg[2] + fabs(r[2]) * Sc * sg[1];
            SF[6 * b + 4] += fabs(r[2]) * Sc * sg[0] + fabs(r[0]) * Sc * sg[2];
            SF[6 * b + 5] += fabs(r[0]) * Sc * sg[1] + fabs(r[1]) * Sc * sg[0];
        }
    }
    for (int32_t b = 0; b < w->nr; ++b) {
        or_rigid *s = &w->bs[b];
        const double *Iv = w->Iwinv + 9 * b, *tq = F + 6 * b + 3;
        for (int a = 0; a < 3; ++a) {
            s->vel[a] += w->dt * F[6 * b + a] / s->mass;
            s->omega[a] += w->dt * (Iv[3 * a] * tq[0] + Iv[3 * a + 1] * tq[1] + Iv[3 * a + 2] * tq[2]);
            w->F[3 * b + a] += F[6 * b + a];
            w->T[3 * b + a] += F[6 * b + 3 + a];
            w->SF[3 * b + a] += SF[6 * b + a];
            w->ST[3 * b + a] += SF[6 * b + 3 + a];
        }
    }
    body_boundary_velocities(w);
    free(F);
    free(SF);
}

static void pressure_update(const world *w, const double *kappa, const double *Skappa, double *v, double *Sv) {
    pressure_update_den(w, kappa, Skappa, w->rho, v, Sv);
    couple_pass((world *)w, kappa, Skappa, w->rho);
}

/* largest clamped (compression-only) deviation */
static double max_pos(const double *a, int64_t n) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (a[i] > m) m = a[i];
    return m;
}

/* mean over fluid particles of a clamped (compression-only) deviation */
static double mean_pos(const double *a, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] > 0.0 ? a[i] : 0.0;
    return n > 0 ? s / (double)n : 0.0;
}
static double mean_abs(const double *a, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += fabs(a[i]);
    return n > 0 ? s / (double)n : 0.0;
}

/* ---- implicit viscosity, Eqs. (16)-(19) --------------------------------- */
/* (A v)_i = sum_j 2(d+2) mu mbar/(rho_i rho_j) gradW_ij (x_ij.(v_i - v_j)) /
 *           (|x_ij|^2 + 0.01 h^2),  mbar = m, mu = nu rho0 (reading of Eq. 19) */
static void visc_A(const world *w, double mu, const double *v, double *Av) {
    const double m = w->m, h = w->h;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < w->nf; ++i) {
        double acc[3] = {0, 0, 0};
        FOR_F(i, e) {
            int64_t j = w->ff.idx[e];
            double x[3], gw[3];
            xij_f(w, i, j, x);
            or_gradW(x, h, gw);
            double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            double c = 2.0 * (3 + 2) * mu * m / (w->rho[i] * w->rho[j]) / (r2 + 0.01 * h * h);
            double xv = x[0] * (v[3 * i] - v[3 * j]) + x[1] * (v[3 * i + 1] - v[3 * j + 1]) +
                        x[2] * (v[3 * i + 2] - v[3 * j + 2]);
            for (int a = 0; a < 3; ++a) acc[a] += c * xv * gw[a];
        }
        for (int a = 0; a < 3; ++a) Av[3 * i + a] = acc[a];
    }
}

/* M v = v - dt A v */
static void visc_M(const world *w, double mu, const double *v, double *Mv) {
    visc_A(w, mu, v, Mv);
    for (int64_t i = 0; i < 3 * w->nf; ++i) Mv[i] = v[i] - w->dt * Mv[i];
}

/* public: one application of M = I - dt A (for the parity of the mat-vec) */
static void inv3(const double M[9], double I[9]) {
    double a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5], g = M[6], hh = M[7], k = M[8];
    double A = e * k - f * hh, B = -(d * k - f * g), C = d * hh - e * g;
    double det = a * A + b * B + c * C;
    double id = 1.0 / det;
    I[0] = A * id; I[1] = -(b * k - c * hh) * id; I[2] = (b * f - c * e) * id;
    I[3] = B * id; I[4] = (a * k - c * g) * id;    I[5] = -(a * f - c * d) * id;
    I[6] = C * id; I[7] = -(a * hh - b * g) * id;  I[8] = (a * e - b * d) * id;
}

/* 3x3 diagonal blocks of M: I + dt sum_j c_ij (-gradW_ij) x_ij^T */
static void visc_block_inverse(const world *w, double mu, double *Pinv) {
    const double m = w->m, h = w->h;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < w->nf; ++i) {
        double B[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        FOR_F(i, e) {
            int64_t j = w->ff.idx[e];
            double x[3], gw[3];
            xij_f(w, i, j, x);
            or_gradW(x, h, gw);
            double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            double c = 2.0 * (3 + 2) * mu * m / (w->rho[i] * w->rho[j]) / (r2 + 0.01 * h * h);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) B[3 * a + b] -= w->dt * c * gw[a] * x[b];
        }
        inv3(B, Pinv + 9 * i);
    }
}

static double dot(const double *a, const double *b, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Preconditioned CG (block Jacobi) from the start value x (on entry), stop at
 * |r| <= tol |b| */
static void visc_cg(world *w, double mu, const double *b, double *x, int32_t *iters, double *resid) {
    int64_t n3 = 3 * w->nf;
    size_t sz = sizeof(double) * (n3 ? n3 : 1);
    double *r = malloc(sz), *z = malloc(sz), *pp = malloc(sz), *Ap = malloc(sz);
    double *Pinv = malloc(sizeof(double) * 9 * (w->nf ? w->nf : 1));
    visc_block_inverse(w, mu, Pinv);
    visc_M(w, mu, x, Ap);
    for (int64_t i = 0; i < n3; ++i) r[i] = b[i] - Ap[i];
    for (int64_t i = 0; i < w->nf; ++i)
        for (int a = 0; a < 3; ++a)
            z[3 * i + a] = Pinv[9 * i + 3 * a] * r[3 * i] + Pinv[9 * i + 3 * a + 1] * r[3 * i + 1] +
                           Pinv[9 * i + 3 * a + 2] * r[3 * i + 2];
    memcpy(pp, z, sz);
    double rz = dot(r, z, n3), bn = sqrt(dot(b, b, n3));
    int32_t it = 0;
    double rn = sqrt(dot(r, r, n3));
    while (rn > w->p->cg_tol * bn && it < w->p->cg_max_iters) {
        visc_M(w, mu, pp, Ap);
        double a = rz / dot(pp, Ap, n3);
        for (int64_t i = 0; i < n3; ++i) { x[i] += a * pp[i]; r[i] -= a * Ap[i]; }
        for (int64_t i = 0; i < w->nf; ++i)
            for (int q = 0; q < 3; ++q)
                z[3 * i + q] = Pinv[9 * i + 3 * q] * r[3 * i] + Pinv[9 * i + 3 * q + 1] * r[3 * i + 1] +
                               Pinv[9 * i + 3 * q + 2] * r[3 * i + 2];
        double rz2 = dot(r, z, n3);
        double beta = rz2 / rz;
        rz = rz2;
        for (int64_t i = 0; i < n3; ++i) pp[i] = z[i] + beta * pp[i];
        rn = sqrt(dot(r, r, n3));
        ++it;
    }
    *iters = it;
    *resid = bn > 0 ? rn / bn : 0.0;
    free(r); free(z); free(pp); free(Ap); free(Pinv);
}

/* ---- the whole step ------------------------------------------------------ */
/* PCISPH stiffness factor (Sec. 3.4.2 names PCISPH; its delta is taken from
 * the predictive-corrective method, in our reading).  delta = 1 / (beta sum_j
 * |gradW_j|^2) with beta = 2 (dt m / rho0)^2, summed once over a prototype
 * particle inside a filled lattice of spacing 2r (its sum_j gradW_j vanishes
 * by symmetry).  In the stiffness form of the density solve, kappa_i = p_i /
 * rho_i = (rho*_i - rho0) c / (rho_i dt^2) with
 *     c = rho0^2 / (2 sum_j |m gradW_j|^2).                                  */
double or_pcisph_factor(const or_params *p) {
    const double s = 2.0 * p->r, h = p->h;
    const double m = p->rho0 * s * s * s;
    const int n = (int)ceil(h / s);
    double sum = 0.0;
    for (int a = -n; a <= n; ++a)
        for (int b = -n; b <= n; ++b)
            for (int c = -n; c <= n; ++c) {
                const double d = s * sqrt((double)(a * a + b * b + c * c));
                if (d == 0.0 || d >= h) continue;
                const double g = m * or_dWdr(d, h);
                sum += g * g;
            }
    return p->rho0 * p->rho0 / (2.0 * sum);
}

/* ------------------------------------------------------------------------ */
/* Rigid contact (our model; the paper leaves rigid dynamics to PyBullet,     */
/* Sec. 4.2).  Bodies touch through their own sample points (their Akinci     */
/* boundary particles): a point within one sampling spacing s = 2r of the     */
/* interior shrunk by r (the tank), or within 2s of another body's point, is  */
/* a contact with normal n (the inward axis, or from the other point to this  */
/* one) and gap g (its distance to the plane, or the points' distance minus   */
/* s).  Frictionless and without restitution, each contact asks that the      */
/* point not close more than its gap within the step: v_n >= -g / dt, v_n the */
/* relative normal velocity at the point.  Normal impulses lambda >= 0 are    */
/* found by projected Gauss-Seidel, 30 sweeps in a fixed order (tank contacts */
/* by body, point, axis, side; then body pairs a < b by point of a and point  */
/* of b), on the velocities the step gave the bodies, at the pose of the step's */
/* start.                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct rc_contact {
    int32_t a, b;              /* bodies (b = -1: the tank) */
    double n[3], ra[3], rb[3]; /* normal, lever arms from the centres */
    double bias, K, lam;
} rc_contact;

static void rc_push(rc_contact **c, int64_t *n, int64_t *cap, rc_contact v) {
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 256;
        *c = realloc(*c, sizeof(rc_contact) * (size_t)*cap);
    }
    (*c)[(*n)++] = v;
}

static void rc_apply(or_rigid *s, const double *Iv, const double r[3], const double n[3], double lam) {
    double rn[3];
    cross(r, n, rn);
    for (int a = 0; a < 3; ++a) {
        s->vel[a] += lam * n[a] / s->mass;
        s->omega[a] += lam * (Iv[3 * a] * rn[0] + Iv[3 * a + 1] * rn[1] + Iv[3 * a + 2] * rn[2]);
    }
}

/* normal velocity of body s at lever arm r */
static double rc_vn(const or_rigid *s, const double r[3], const double n[3]) {
    double wr[3];
    cross(s->omega, r, wr);
    return (s->vel[0] + wr[0]) * n[0] + (s->vel[1] + wr[1]) * n[1] + (s->vel[2] + wr[2]) * n[2];
}

/* 1/M + (r x n) . I^-1 (r x n) */
static double rc_inv_mass(const or_rigid *s, const double *Iv, const double r[3], const double n[3]) {
    double rn[3], t[3];
    cross(r, n, rn);
    for (int a = 0; a < 3; ++a) t[a] = Iv[3 * a] * rn[0] + Iv[3 * a + 1] * rn[1] + Iv[3 * a + 2] * rn[2];
    return 1.0 / s->mass + rn[0] * t[0] + rn[1] * t[1] + rn[2] * t[2];
}

static void rigid_contacts(const or_params *p, const or_in *in, double dt, or_rigid *bs) {
    const int32_t nr = p->n_rigid;
    const int64_t nb = in->nb;
    const double s2 = 2.0 * p->r;
    if (nr <= 0) return;
    double *P = malloc(sizeof(double) * 3 * (size_t)(nb ? nb : 1));
    double *Iv = calloc((size_t)(9 * nr), sizeof(double));
    double *reach = calloc((size_t)nr, sizeof(double));
    for (int32_t b = 0; b < nr; ++b) {
        double R[9];
        quat_to_R(bs[b].quat, R);
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                for (int q = 0; q < 3; ++q) Iv[9 * b + 3 * a + c] += R[3 * a + q] / bs[b].inertia[q] * R[3 * c + q];
        for (int64_t k = 0; k < nb; ++k) {
            if (in->body[k] != b) continue;
            const double *l = in->local + 3 * k;
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                P[3 * k + a] = bs[b].com[a] + (R[3 * a] * l[0] + R[3 * a + 1] * l[1] + R[3 * a + 2] * l[2]);
                r2 += l[a] * l[a];
            }
            if (sqrt(r2) > reach[b]) reach[b] = sqrt(r2);
        }
    }
    rc_contact *cs = NULL;
    int64_t nc = 0, cap = 0;
    for (int32_t b = 0; b < nr; ++b)
        for (int64_t k = 0; k < nb; ++k) {
            if (in->body[k] != b) continue;
            for (int a = 0; a < 3; ++a)
                for (int side = 0; side < 2; ++side) {
                    const double plane = side == 0 ? p->domain_min[a] + p->r : p->domain_max[a] - p->r;
                    const double g = side == 0 ? P[3 * k + a] - plane : plane - P[3 * k + a];
                    if (g >= s2) continue;
                    rc_contact c;
                    memset(&c, 0, sizeof(c));
                    c.a = b; c.b = -1;
                    c.n[a] = side == 0 ? 1.0 : -1.0;
                    for (int q = 0; q < 3; ++q) c.ra[q] = P[3 * k + q] - bs[b].com[q];
                    c.bias = -g / dt;
                    c.K = rc_inv_mass(&bs[b], Iv + 9 * b, c.ra, c.n);
                    rc_push(&cs, &nc, &cap, c);
                }
        }
    for (int32_t a = 0; a < nr; ++a)
        for (int32_t b = a + 1; b < nr; ++b) {
            double dc = 0.0;
            for (int q = 0; q < 3; ++q) dc += (bs[a].com[q] - bs[b].com[q]) * (bs[a].com[q] - bs[b].com[q]);
            if (sqrt(dc) >= reach[a] + reach[b] + 2.0 * s2) continue;
            for (int64_t k = 0; k < nb; ++k) {
                if (in->body[k] != a) continue;
                for (int64_t j = 0; j < nb; ++j) {
                    if (in->body[j] != b) continue;
                    double d[3], dd = 0.0;
                    for (int q = 0; q < 3; ++q) { d[q] = P[3 * k + q] - P[3 * j + q]; dd += d[q] * d[q]; }
                    dd = sqrt(dd);
                    if (!(dd < 2.0 * s2) || dd == 0.0) continue;
                    rc_contact c;
                    memset(&c, 0, sizeof(c));
                    c.a = a; c.b = b;
                    for (int q = 0; q < 3; ++q) {
                        c.n[q] = d[q] / dd;
                        c.ra[q] = P[3 * k + q] - bs[a].com[q];
                        c.rb[q] = P[3 * j + q] - bs[b].com[q];
                    }
                    c.bias = -(dd - s2) / dt;
                    c.K = rc_inv_mass(&bs[a], Iv + 9 * a, c.ra, c.n) + rc_inv_mass(&bs[b], Iv + 9 * b, c.rb, c.n);
                    rc_push(&cs, &nc, &cap, c);
                }
            }
        }
    for (int sweep = 0; sweep < 30; ++sweep)
        for (int64_t i = 0; i < nc; ++i) {
            rc_contact *c = &cs[i];
            double vn = rc_vn(&bs[c->a], c->ra, c->n);
            if (c->b >= 0) vn -= rc_vn(&bs[c->b], c->rb, c->n);
            double lam = c->lam + (c->bias - vn) / c->K;
            if (lam < 0.0) lam = 0.0;
            const double dl = lam - c->lam;
            c->lam = lam;
            if (dl == 0.0) continue;
            rc_apply(&bs[c->a], Iv + 9 * c->a, c->ra, c->n, dl);
            if (c->b >= 0) rc_apply(&bs[c->b], Iv + 9 * c->b, c->rb, c->n, -dl);
        }
    free(cs); free(P); free(Iv); free(reach);
}

int or_step(const or_params *p, const or_in *in, or_out *out) {
    if (p->solver == 2 && p->warm_start == 2) return -2;   /* the learned start is DFSPH's */
    if (in->nf < 0 || in->nb < 0) return -3;
    world W_, *w = &W_;
    memset(w, 0, sizeof(*w));
    const int64_t nf = in->nf, nb = in->nb, n3 = 3 * nf;
    const size_t s1 = sizeof(double) * (nf ? nf : 1), s3 = 3 * s1;
    w->p = p; w->nf = nf; w->nb = nb;
    w->h = p->h;
    w->m = p->rho0 * (2.0 * p->r) * (2.0 * p->r) * (2.0 * p->r);
    w->k0 = or_W(0.0, p->h);

    /* -- 1. time step: fixed, or CFL from the input velocities.  Reading:
     *    dt = fl32(min(dt_max, lambda * 2r / sqrt(max_i fl32(|v_i|^2)))). */
    if (p->cfl_lambda > 0.0) {
        float vmax2 = 0.0f;
        for (int64_t i = 0; i < nf; ++i) {
            const float *vi = in->vf + 3 * i;
            float a = vi[0] * vi[0], b = vi[1] * vi[1], c = vi[2] * vi[2];
            float s = a + b;
            s = s + c;
            if (s > vmax2) vmax2 = s;
        }
        double dt = p->dt_max;
        if (vmax2 > 0.0f) {
            double c = p->cfl_lambda * (2.0 * p->r) / sqrt((double)vmax2);
            if (c < dt) dt = c;
        }
        w->dt = (double)(float)dt;
    } else {
        w->dt = (double)(float)p->dt_max;
    }
    const double dt = w->dt;
    out->dt = dt;

    /* -- 2. keys, sort and neighbour sets (FP32 predicate) */
    or_grid g;
    or_grid_make(p->h, p->domain_min, p->domain_max, &g);
    uint32_t *perm_f, *start_f, *perm_b, *start_b;
    float *xs_f, *xs_b;
    sort_points(&g, in->xf, nf, &perm_f, &xs_f, &start_f);
    sort_points(&g, in->xb, nb, &perm_b, &xs_b, &start_b);
    build_csr(&g, xs_f, perm_f, nf, xs_f, perm_f, start_f, nf, 1, in->brute_force, &w->ff);
    build_csr(&g, xs_f, perm_f, nf, xs_b, perm_b, start_b, nb, 0, in->brute_force, &w->fb);
    csr bb;
    build_csr(&g, xs_b, perm_b, nb, xs_b, perm_b, start_b, nb, 1, in->brute_force, &bb);

    w->x = malloc(s3); w->v = malloc(s3); w->Sv = malloc(s3);
    for (int64_t i = 0; i < n3; ++i) { w->x[i] = in->xf[i]; w->v[i] = in->vf[i]; w->Sv[i] = fabs(w->v[i]); }
    size_t sb = sizeof(double) * 3 * (nb ? nb : 1);
    w->xb = malloc(sb); w->vb = malloc(sb); w->psi = malloc(sb / 3);
    for (int64_t i = 0; i < 3 * nb; ++i) { w->xb[i] = in->xb[i]; w->vb[i] = in->vb[i]; }

    /* -- 3. Psi, Eq. (11) */
    boundary_psi(p, w->xb, nb, &bb, w->psi);

    /* bodies during the step (strong coupling): their velocities change
     * with every pressure pass; the pose (and so the world inertia) stays */
    w->nr = p->n_rigid;
    w->strong = p->rigid_coupling == 1 && p->n_rigid > 0;
    w->body = in->body;
    w->xb32 = in->xb;
    const size_t snr = (size_t)(p->n_rigid > 0 ? p->n_rigid : 1);
    w->bs = malloc(sizeof(or_rigid) * snr);
    w->Iw = calloc(9 * snr, sizeof(double));
    w->Iwinv = calloc(9 * snr, sizeof(double));
    w->F = calloc(3 * snr, sizeof(double)); w->T = calloc(3 * snr, sizeof(double));
    w->SF = calloc(3 * snr, sizeof(double)); w->ST = calloc(3 * snr, sizeof(double));
    for (int32_t b = 0; b < p->n_rigid; ++b) {
        w->bs[b] = in->rigid[b];
        double R[9];
        quat_to_R(in->rigid[b].quat, R);
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                for (int q = 0; q < 3; ++q) {
                    w->Iw[9 * b + 3 * a + c] += R[3 * a + q] * in->rigid[b].inertia[q] * R[3 * c + q];
                    w->Iwinv[9 * b + 3 * a + c] += R[3 * a + q] / in->rigid[b].inertia[q] * R[3 * c + q];
                }
    }

    /* -- 4. density (Eq. 12) and alpha */
    w->rho = malloc(s1); w->alpha = malloc(s1); w->Salpha = malloc(s1);
    density_alpha(w);
    const int dfsph = p->solver == 0, pcisph = p->solver == 2;
    if (pcisph) {
        /* PCISPH: the density solve's factor is c / rho_i instead of
         * the DFSPH alpha; it is reported in its place */
        const double c = or_pcisph_factor(p);
        for (int64_t i = 0; i < nf; ++i) {
            w->alpha[i] = c / w->rho[i];
            w->Salpha[i] = w->alpha[i];
        }
    }

    double *v_in = malloc(s3);
    memcpy(v_in, w->v, s3);
    double *d = malloc(s1), *Sd = malloc(s1), *kap = malloc(s1), *Skap = malloc(s1);
    /* the density change rate of the step's input velocity (before any
     * pressure of this step), a feature of the learned warm start */
    double *d_in = malloc(s1), *Sd_in = malloc(s1);
    divergence(w, w->v, w->Sv, d_in, Sd_in);
    double *Kv = malloc(s1), *SKv = malloc(s1), *K = malloc(s1), *SK = malloc(s1);
    double *kappa_last = calloc((size_t)(nf ? nf : 1), sizeof(double));
    double *Skappa_last = calloc((size_t)(nf ? nf : 1), sizeof(double));

    int32_t lv = 0;
    double err_v = 0.0, S_err_v = 0.0;
    if (dfsph) {
        /* -- 5. divergence-free solve (Eq. 10 with Algorithm 2).  Warm start
         *    (Algorithm 2 leaves it open): zero (ZERO), or kappa/rho = warm_factor Kv_prev / rho_prev,
         *    the previous step's stiffness over its own density (PREVIOUS,
         *    LEARNED); it accumulates as Kv0 = that times the current rho. */
        double *rp = malloc(s1);
        for (int64_t i = 0; i < nf; ++i) {
            rp[i] = in->rho_prev ? (double)in->rho_prev[i] : p->rho0;
            Kv[i] = p->warm_start == 0 ? 0.0 : p->warm_factor * (double)in->Kv[i];
            SKv[i] = fabs(Kv[i]);
        }
        if (p->warm_start != 0) {
            pressure_update_den(w, Kv, SKv, rp, w->v, w->Sv);
            couple_pass(w, Kv, SKv, rp);
        }
        for (int64_t i = 0; i < nf; ++i) {
            Kv[i] = Kv[i] / rp[i] * w->rho[i];
            SKv[i] = fabs(Kv[i]);
        }
        free(rp);
        divergence(w, w->v, w->Sv, d, Sd);
        err_v = dt / p->rho0 * mean_pos(d, nf);
        S_err_v = dt / p->rho0 * mean_abs(Sd, nf);
        out->err_div_hist[0] = err_v;
        for (;;) {
            int go = p->forced_div >= 0 ? (lv < p->forced_div) : (err_v > p->eta_divergence && lv < p->max_iters);
            if (!go) break;
            for (int64_t i = 0; i < nf; ++i) {
                double dp = d[i] > 0.0 ? d[i] : 0.0;
                kap[i] = dp * w->alpha[i] / dt;
                Skap[i] = (Sd[i] * w->alpha[i] + dp * w->Salpha[i]) / dt;
            }
            pressure_update(w, kap, Skap, w->v, w->Sv);
            for (int64_t i = 0; i < nf; ++i) { Kv[i] += kap[i]; SKv[i] += Skap[i]; }
            ++lv;
            divergence(w, w->v, w->Sv, d, Sd);
            err_v = dt / p->rho0 * mean_pos(d, nf);
            S_err_v = dt / p->rho0 * mean_abs(Sd, nf);
            if (lv < 128) out->err_div_hist[lv] = err_v;
        }
    } else {
        /* WCSPH and PCISPH have no divergence solve */
        for (int64_t i = 0; i < nf; ++i) { Kv[i] = 0.0; SKv[i] = 0.0; d[i] = 0.0; Sd[i] = 0.0; }
        out->err_div_hist[0] = 0.0;
    }
    out->iters_div = lv;
    out->err_div = err_v;
    out->S_err_div = S_err_v;
    out->converged_div = err_v <= p->eta_divergence;

    /* the bodies' own non-pressure accelerations (strong coupling): gravity
     * and the gyroscopic term, between the two solves as for the fluid */
    if (w->strong) {
        for (int32_t b = 0; b < p->n_rigid; ++b) {
            or_rigid *s = &w->bs[b];
            const double *Iw = w->Iw + 9 * b, *Iv = w->Iwinv + 9 * b;
            double L[3], gy[3];
            for (int a = 0; a < 3; ++a) L[a] = Iw[3 * a] * s->omega[0] + Iw[3 * a + 1] * s->omega[1] + Iw[3 * a + 2] * s->omega[2];
            cross(s->omega, L, gy);
            for (int a = 0; a < 3; ++a) {
                s->vel[a] += dt * p->gravity[a];
                s->omega[a] -= dt * (Iv[3 * a] * gy[0] + Iv[3 * a + 1] * gy[1] + Iv[3 * a + 2] * gy[2]);
            }
        }
        body_boundary_velocities(w);
    }

    /* -- 6. non-pressure accelerations (Algorithm 1, first two lines):
     *    gravity plus XSPH, Eq. (15), or the implicit solve of Eqs. (16)-(19). */
    double *vs = malloc(s3), *Svs = malloc(s3);
    const double *gr = p->gravity;
    out->cg_iters = 0;
    out->cg_resid = 0.0;
    if (p->visc_model == 1) {
        /* XSPH: v*_i = v_i + dt g + eps sum_F (m/rho_j)(v_j - v_i) W_ij */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nf; ++i) {
            double acc[3] = {0, 0, 0}, Sacc[3] = {0, 0, 0};
            FOR_F(i, e) {
                int64_t j = w->ff.idx[e];
                double x[3];
                xij_f(w, i, j, x);
                double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                double Wij = or_W(r, w->h), SW = W_scale(r, w->h);
                for (int a = 0; a < 3; ++a) {
                    acc[a] += w->m / w->rho[j] * (w->v[3 * j + a] - w->v[3 * i + a]) * Wij;
                    Sacc[a] += w->m / w->rho[j] * (w->Sv[3 * j + a] + w->Sv[3 * i + a]) * SW;
                }
            }
            for (int a = 0; a < 3; ++a) {
                vs[3 * i + a] = w->v[3 * i + a] + dt * gr[a] + p->visc * acc[a];
                Svs[3 * i + a] = w->Sv[3 * i + a] + dt * fabs(gr[a]) + p->visc * Sacc[a];
            }
        }
    } else if (p->visc_model == 2) {
        /* Eq. (15): lap v_i = 2(d+2) sum_F (m/rho_j) (v_ij.x_ij)/(|x_ij|^2+0.01h^2) gradW_ij */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nf; ++i) {
            double acc[3] = {0, 0, 0}, Sacc[3] = {0, 0, 0};
            FOR_F(i, e) {
                int64_t j = w->ff.idx[e];
                double x[3], gw[3], sg[3];
                xij_f(w, i, j, x);
                or_gradW(x, w->h, gw);
                gradW_scale(x, w->h, sg);
                double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
                double den = r2 + 0.01 * w->h * w->h;
                double vx = 0.0, Svx = 0.0;
                for (int a = 0; a < 3; ++a) {
                    vx += (w->v[3 * i + a] - w->v[3 * j + a]) * x[a];
                    Svx += (w->Sv[3 * i + a] + w->Sv[3 * j + a]) * fabs(x[a]);
                }
                for (int a = 0; a < 3; ++a) {
                    acc[a] += w->m / w->rho[j] * vx / den * gw[a];
                    Sacc[a] += w->m / w->rho[j] * Svx / den * sg[a];
                }
            }
            for (int a = 0; a < 3; ++a) {
                vs[3 * i + a] = w->v[3 * i + a] + dt * gr[a] + dt * p->visc * 2.0 * (3 + 2) * acc[a];
                Svs[3 * i + a] = w->Sv[3 * i + a] + dt * fabs(gr[a]) + dt * p->visc * 2.0 * (3 + 2) * Sacc[a];
            }
        }
    } else if (p->visc_model == 3) {
        double *b = malloc(s3);
        for (int64_t i = 0; i < nf; ++i)
            for (int a = 0; a < 3; ++a) b[3 * i + a] = w->v[3 * i + a] + dt * gr[a];
        /* start value (Sec. 3.6 gives none): x0 = b + cg_warm_factor times the previous
         * step's correction v* - b */
        for (int64_t i = 0; i < n3; ++i)
            vs[i] = b[i] + (in->dvisc ? p->cg_warm_factor * (double)in->dvisc[i] : 0.0);
        visc_cg(w, p->visc * p->rho0, b, vs, &out->cg_iters, &out->cg_resid);
        if (out->dvisc)
            for (int64_t i = 0; i < n3; ++i) out->dvisc[i] = vs[i] - b[i];
        /* the CG result is compared by its residual, so its scale is its size */
        for (int64_t i = 0; i < n3; ++i) Svs[i] = w->Sv[i] + fabs(vs[i]);
        free(b);
    } else {
        for (int64_t i = 0; i < nf; ++i)
            for (int a = 0; a < 3; ++a) {
                vs[3 * i + a] = w->v[3 * i + a] + dt * gr[a];
                Svs[3 * i + a] = w->Sv[3 * i + a] + dt * fabs(gr[a]);
            }
    }
    memcpy(w->v, vs, s3);
    memcpy(w->Sv, Svs, s3);

    /* -- 7. warm start of the density solve (Algorithm 2, "initialize p^l"):
     *    K0 = 0, warm_factor * K_prev, or the learned prediction
     *    max(0, y alpha rho0 / dt^2) of the step's final stiffness, y = MLP of
     *    five dimensionless features; the target is K_final dt^2 / (alpha rho0).
     *    Features: (rho - rho0)/rho0, dt d/rho0 with d the density change
     *    rate (Eq. 9, DFSPH form) of the step's input velocity, before any
     *    pressure of this step, (n_f + n_b)/26, K_prev dt^2/(alpha rho0),
     *    alpha/alpha_ref. */
    const double alpha_ref = 2.35376 * (2.0 * p->r) * (2.0 * p->r) / p->rho0;
    double *feat = NULL, *Sfeat = NULL;
    if (dfsph && (p->warm_start == 2 || out->features)) {
        feat = malloc(sizeof(double) * 5 * (nf ? nf : 1));
        Sfeat = malloc(sizeof(double) * 5 * (nf ? nf : 1));
        for (int64_t i = 0; i < nf; ++i) {
            int64_t n_i = (w->ff.start[i + 1] - w->ff.start[i]) + (w->fb.start[i + 1] - w->fb.start[i]);
            double a = w->alpha[i];
            feat[5 * i + 0] = (w->rho[i] - p->rho0) / p->rho0;
            feat[5 * i + 1] = dt * d_in[i] / p->rho0;
            feat[5 * i + 2] = (double)n_i / 26.0;
            feat[5 * i + 3] = a > 0.0 ? (double)in->K[i] * dt * dt / (a * p->rho0) : 0.0;
            feat[5 * i + 4] = a / alpha_ref;
            {
                double *S = Sfeat + 5 * i;
                S[0] = (w->rho[i] + p->rho0) / p->rho0;
                S[1] = dt * Sd_in[i] / p->rho0;
                S[2] = 0.0;
                S[3] = a > 0.0 ? fabs(feat[5 * i + 3]) * (1.0 + w->Salpha[i] / a) : 0.0;
                S[4] = w->Salpha[i] / alpha_ref;
            }
        }
        if (out->features) memcpy(out->features, feat, sizeof(double) * 5 * nf);
        if (out->S_features) memcpy(out->S_features, Sfeat, sizeof(double) * 5 * nf);
    }
    for (int64_t i = 0; i < nf; ++i) {
        K[i] = p->warm_start == 0 ? 0.0 : p->warm_factor * (double)in->K[i];
        SK[i] = fabs(K[i]);
    }
    if (dfsph && p->warm_start == 2) {
        double *y = malloc(2 * s1);
        in->mlp(feat, Sfeat, nf, y, in->mlp_user);
        for (int64_t i = 0; i < nf; ++i) {
            double k0 = y[i] * w->alpha[i] * p->rho0 / (dt * dt);
            K[i] = k0 > 0.0 ? k0 : 0.0;
            SK[i] = fabs(k0) + (y[nf + i] + fabs(y[i]) * w->Salpha[i] / w->alpha[i]) * w->alpha[i] * p->rho0 / (dt * dt);
        }
        free(y);
    }
    if ((dfsph || pcisph) && p->warm_start != 0) pressure_update(w, K, SK, w->v, w->Sv);

    /* -- 8. constant-density solve (Eqs. 8, 9 with Eq. 7, Algorithm 2):
     *    rho*_i = rho_i + dt d_i(v*), kappa_i = max(rho*_i - rho0, 0) alpha_i / dt^2,
     *    with PCISPH's c / rho_i in place of alpha_i.  The error of
     *    Algorithm 2 is the mean compression; with eta_density_max > 0 the
     *    solve also iterates while the largest compression exceeds it. */
    double *rs = malloc(s1), *Srs = malloc(s1);
    double err_d, S_err_d, err_dmax = 0.0;
#define PREDICT_DENSITY()                                                   \
    do {                                                                    \
        divergence(w, w->v, w->Sv, d, Sd);                                  \
        for (int64_t i = 0; i < nf; ++i) {                                  \
            rs[i] = w->rho[i] + dt * d[i] - p->rho0;                        \
            Srs[i] = w->rho[i] + dt * Sd[i] + p->rho0;                      \
        }                                                                   \
        err_d = mean_pos(rs, nf) / p->rho0;                                 \
        S_err_d = mean_abs(Srs, nf) / p->rho0;                              \
        err_dmax = max_pos(rs, nf) / p->rho0;                               \
    } while (0)
    int32_t ld = 0;
    if (dfsph || pcisph) {
        PREDICT_DENSITY();
        out->err_dens_hist[0] = err_d;
        out->err_dens_max_hist[0] = err_dmax;
        for (;;) {
            const int above = err_d > p->eta_density || (p->eta_density_max > 0.0 && err_dmax > p->eta_density_max);
            int go = p->forced_dens >= 0 ? (ld < p->forced_dens) : (above && ld < p->max_iters);
            if (!go) break;
            for (int64_t i = 0; i < nf; ++i) {
                double e = rs[i] > 0.0 ? rs[i] : 0.0;
                kap[i] = e * w->alpha[i] / (dt * dt);
                Skap[i] = (Srs[i] * w->alpha[i] + e * w->Salpha[i]) / (dt * dt);
            }
            pressure_update(w, kap, Skap, w->v, w->Sv);
            for (int64_t i = 0; i < nf; ++i) {
                K[i] += kap[i]; SK[i] += Skap[i];
                kappa_last[i] = kap[i]; Skappa_last[i] = Skap[i];
            }
            ++ld;
            PREDICT_DENSITY();
            if (ld < 128) {
                out->err_dens_hist[ld] = err_d;
                out->err_dens_max_hist[ld] = err_dmax;
            }
        }
    } else {
        /* -- 8w. WCSPH (Sec. 3.4.1): the equation of state
         *    p_i = k ((rho_i/rho0)^gamma - 1), clamped at zero (no tension), then
         *    one pressure pass on v* with kappa_i = p_i / rho_i (p/rho^2 =
         *    kappa/rho).  The reported error is the mean compression of rho itself. */
        for (int64_t i = 0; i < nf; ++i) {
            const double ratio = w->rho[i] / p->rho0;
            const double pw = pow(ratio, p->wcsph_gamma);
            double pr = p->wcsph_k * (pw - 1.0);
            if (pr < 0.0) pr = 0.0;
            kap[i] = pr / w->rho[i];
            /* scale: the two terms of the difference, and rho's own rounding
             * through the exponent */
            Skap[i] = p->wcsph_k * (pw + 1.0) * (1.0 + p->wcsph_gamma) / w->rho[i];
            K[i] = kap[i]; SK[i] = Skap[i];
            kappa_last[i] = kap[i]; Skappa_last[i] = Skap[i];
            rs[i] = w->rho[i] - p->rho0;
            Srs[i] = w->rho[i] + p->rho0;
        }
        pressure_update(w, kap, Skap, w->v, w->Sv);
        err_d = mean_pos(rs, nf) / p->rho0;
        S_err_d = mean_abs(Srs, nf) / p->rho0;
        out->err_dens_hist[0] = err_d;
    }
#undef PREDICT_DENSITY
    out->iters_dens = ld;
    out->err_dens = err_d;
    out->S_err_dens = S_err_d;
    out->err_dens_max = (dfsph || pcisph) && p->eta_density_max > 0.0 ? err_dmax : 0.0;
    out->converged_dens = err_d <= p->eta_density && (p->eta_density_max <= 0.0 || !(dfsph || pcisph) ||
                                                      err_dmax <= p->eta_density_max);

    /* -- 9. reaction on the rigid bodies (Eq. 14): the pressure impulses of
     *    every pass of this step divided by dt, i.e. with K_tot = Kv + K:
     *    F_b = sum_i sum_{k in b} m Psi_k (K_tot_i / rho_i) gradW_ik,
     *    tau_b = sum (x_k - c_b) x F_ik. */
    for (int32_t b = 0; b < p->n_rigid; ++b)
        for (int a = 0; a < 3; ++a) {
            out->force[3 * b + a] = 0.0; out->torque[3 * b + a] = 0.0;
            if (out->S_force) { out->S_force[3 * b + a] = 0.0; out->S_torque[3 * b + a] = 0.0; }
        }
    for (int64_t i = 0; i < nf && !w->strong; ++i) {
        FOR_B(i, e) {
            int64_t k = w->fb.idx[e];
            int32_t b = in->body[k];
            if (b < 0) continue;
            double x[3], gw[3], sg[3], F[3], SF[3], rr[3], t[3];
            xij_b(w, i, k, x);
            or_gradW(x, w->h, gw);
            gradW_scale(x, w->h, sg);
            double c = w->m * w->psi[k] * (Kv[i] + K[i]) / w->rho[i];
            double Sc = w->m * w->psi[k] * (SKv[i] + SK[i] + fabs(Kv[i] + K[i])) / w->rho[i];
            for (int a = 0; a < 3; ++a) {
                F[a] = c * gw[a]; SF[a] = Sc * sg[a];
                rr[a] = w->xb[3 * k + a] - in->rigid[b].com[a];
            }
            cross(rr, F, t);
            for (int a = 0; a < 3; ++a) { out->force[3 * b + a] += F[a]; out->torque[3 * b + a] += t[a]; }
            if (out->S_force) {
                double ar[3] = {fabs(rr[0]), fabs(rr[1]), fabs(rr[2])};
                out->S_force[3 * b + 0] += SF[0]; out->S_force[3 * b + 1] += SF[1]; out->S_force[3 * b + 2] += SF[2];
                out->S_torque[3 * b + 0] += ar[1] * SF[2] + ar[2] * SF[1];
                out->S_torque[3 * b + 1] += ar[2] * SF[0] + ar[0] * SF[2];
                out->S_torque[3 * b + 2] += ar[0] * SF[1] + ar[1] * SF[0];
            }
        }
    }

    if (w->strong)   /* the reactions were summed pass by pass */
        for (int32_t b = 0; b < p->n_rigid; ++b)
            for (int a = 0; a < 3; ++a) {
                out->force[3 * b + a] = w->F[3 * b + a];
                out->torque[3 * b + a] = w->T[3 * b + a];
                if (out->S_force) {
                    out->S_force[3 * b + a] = w->SF[3 * b + a];
                    out->S_torque[3 * b + a] = w->ST[3 * b + a];
                }
            }

    /* -- 10. symplectic Euler (Algorithm 1, last two lines): v = v*, x += dt v */
    for (int64_t i = 0; i < nf; ++i) {
        for (int a = 0; a < 3; ++a) {
            double vn = w->v[3 * i + a];
            out->v[3 * i + a] = vn;
            out->S_v[3 * i + a] = w->Sv[3 * i + a];
            out->x[3 * i + a] = w->x[3 * i + a] + dt * vn;
            out->S_x[3 * i + a] = fabs(w->x[3 * i + a]) + dt * w->Sv[3 * i + a];
            out->accel[3 * i + a] = (vn - v_in[3 * i + a]) / dt;
            out->S_accel[3 * i + a] = (w->Sv[3 * i + a] + fabs(v_in[3 * i + a])) / dt;
        }
        out->rho[i] = w->rho[i];
        out->alpha[i] = w->alpha[i];
        out->S_alpha[i] = w->Salpha[i];
        out->K[i] = K[i]; out->S_K[i] = SK[i];
        out->Kv[i] = Kv[i]; out->S_Kv[i] = SKv[i];
        out->kappa[i] = kappa_last[i]; out->S_kappa[i] = Skappa_last[i];
        out->nf_count[i] = (int32_t)(w->ff.start[i + 1] - w->ff.start[i]);
        out->nb_count[i] = (int32_t)(w->fb.start[i + 1] - w->fb.start[i]);
        if (out->target) {
            double a = w->alpha[i];
            out->target[i] = a > 0.0 ? K[i] * dt * dt / (a * p->rho0) : 0.0;
            if (out->S_target)
                out->S_target[i] = a > 0.0 ? (SK[i] + fabs(K[i]) * w->Salpha[i] / a) * dt * dt / (a * p->rho0) : 0.0;
        }
    }
    if (out->psi) memcpy(out->psi, w->psi, sizeof(double) * nb);

    /* -- rigid bodies, FP64: (1) the velocities (weak coupling: the step's
     *    reaction, gravity and the gyroscopic term now; strong: advanced
     *    during the step), (2) rigid contact on those velocities, (3) the
     *    pose; then the boundary particles of the new pose.  Without rigid
     *    contact a stand-in that pushes each body back inside the tank
     *    replaces (2). */
    for (int32_t b = 0; b < p->n_rigid; ++b) {
        or_rigid s = in->rigid[b];
        if (w->strong) {
            for (int a = 0; a < 3; ++a) { s.vel[a] = w->bs[b].vel[a]; s.omega[a] = w->bs[b].omega[a]; }
        } else {
            double R[9], Iw[9], Iwinv[9];
            quat_to_R(s.quat, R);
            /* world inertia R diag(I) R^T and its inverse R diag(1/I) R^T */
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) {
                    Iw[3 * a + c] = 0.0; Iwinv[3 * a + c] = 0.0;
                    for (int q = 0; q < 3; ++q) {
                        Iw[3 * a + c] += R[3 * a + q] * s.inertia[q] * R[3 * c + q];
                        Iwinv[3 * a + c] += R[3 * a + q] / s.inertia[q] * R[3 * c + q];
                    }
                }
            for (int a = 0; a < 3; ++a) s.vel[a] += dt * (out->force[3 * b + a] / s.mass + gr[a]);
            double Lw[3], gyro[3], rhs[3];
            for (int a = 0; a < 3; ++a) Lw[a] = Iw[3 * a] * s.omega[0] + Iw[3 * a + 1] * s.omega[1] + Iw[3 * a + 2] * s.omega[2];
            cross(s.omega, Lw, gyro);
            for (int a = 0; a < 3; ++a) rhs[a] = out->torque[3 * b + a] - gyro[a];
            for (int a = 0; a < 3; ++a)
                s.omega[a] += dt * (Iwinv[3 * a] * rhs[0] + Iwinv[3 * a + 1] * rhs[1] + Iwinv[3 * a + 2] * rhs[2]);
        }
        out->rigid_new[b] = s;
    }
    if (p->rigid_contact == 1) rigid_contacts(p, in, dt, out->rigid_new);
    for (int32_t b = 0; b < p->n_rigid; ++b) {
        or_rigid s = out->rigid_new[b];
        double R[9];
        for (int a = 0; a < 3; ++a) s.com[a] += dt * s.vel[a];
        {
            double qw = s.quat[0], qx = s.quat[1], qy = s.quat[2], qz = s.quat[3];
            double ox = s.omega[0], oy = s.omega[1], oz = s.omega[2];
            double dw = -(ox * qx + oy * qy + oz * qz);
            double dx = ox * qw + (oy * qz - oz * qy);
            double dy = oy * qw + (oz * qx - ox * qz);
            double dz = oz * qw + (ox * qy - oy * qx);
            qw += 0.5 * dt * dw; qx += 0.5 * dt * dx; qy += 0.5 * dt * dy; qz += 0.5 * dt * dz;
            double nq = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            s.quat[0] = qw / nq; s.quat[1] = qx / nq; s.quat[2] = qy / nq; s.quat[3] = qz / nq;
        }
        if (p->rigid_contact != 1) {
            /* tank-contact stand-in: push the body back inside [min + r, max - r]
             * along each axis and drop the velocity component into the wall */
            quat_to_R(s.quat, R);
            for (int a = 0; a < 3; ++a) {
                double lo = 1e300, hi = -1e300;
                for (int64_t k = 0; k < nb; ++k) {
                    if (in->body[k] != b) continue;
                    const double *l = in->local + 3 * k;
                    double xa = s.com[a] + (R[3 * a] * l[0] + R[3 * a + 1] * l[1] + R[3 * a + 2] * l[2]);
                    if (xa < lo) lo = xa;
                    if (xa > hi) hi = xa;
                }
                double wl = p->domain_min[a] + p->r, wh = p->domain_max[a] - p->r;
                if (lo < wl) { s.com[a] += wl - lo; if (s.vel[a] < 0.0) s.vel[a] = 0.0; }
                else if (hi > wh) { s.com[a] -= hi - wh; if (s.vel[a] > 0.0) s.vel[a] = 0.0; }
            }
        }
        out->rigid_new[b] = s;
    }
    for (int64_t k = 0; k < nb; ++k) {
        int32_t b = in->body[k];
        if (b < 0) {
            for (int a = 0; a < 3; ++a) { out->xb_new[3 * k + a] = in->xb[3 * k + a]; out->vb_new[3 * k + a] = in->vb[3 * k + a]; }
            continue;
        }
        const or_rigid *s = &out->rigid_new[b];
        double R[9], xk[3], rr[3], wx[3];
        quat_to_R(s->quat, R);
        const double *l = in->local + 3 * k;
        for (int a = 0; a < 3; ++a) {
            double t = R[3 * a] * l[0] + R[3 * a + 1] * l[1];
            t = t + R[3 * a + 2] * l[2];
            xk[a] = s->com[a] + t;
            out->xb_new[3 * k + a] = (float)xk[a];
        }
        for (int a = 0; a < 3; ++a) rr[a] = (double)out->xb_new[3 * k + a] - s->com[a];
        cross(s->omega, rr, wx);
        for (int a = 0; a < 3; ++a) out->vb_new[3 * k + a] = (float)(s->vel[a] + wx[a]);
    }

    free(feat);
    free(Sfeat);
    free(rs); free(Srs); free(vs); free(Svs);
    free(d_in); free(Sd_in);
    free(v_in); free(d); free(Sd); free(kap); free(Skap); free(Kv); free(SKv); free(K); free(SK);
    free(kappa_last); free(Skappa_last);
    free(w->x); free(w->v); free(w->Sv); free(w->xb); free(w->vb); free(w->psi);
    free(w->rho); free(w->alpha); free(w->Salpha);
    free(w->bs); free(w->Iw); free(w->Iwinv); free(w->F); free(w->T); free(w->SF); free(w->ST);
    csr_free(&w->ff); csr_free(&w->fb); csr_free(&bb);
    free(perm_f); free(start_f); free(xs_f); free(perm_b); free(start_b); free(xs_b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Stand-alone pieces used by the pins                                       */
/* ------------------------------------------------------------------------ */

/* Dense assembly of M = I - dt A (Eq. 18/19) for n <= a few hundred, plus the
 * densities it uses, in id order; M is [3n][3n] row-major. */
int or_visc_dense(const or_params *p, const float *xf, int64_t nf, double dt, double *M, double *rho_out) {
    world W_, *w = &W_;
    memset(w, 0, sizeof(*w));
    w->p = p; w->nf = nf; w->nb = 0; w->h = p->h; w->dt = dt;
    w->m = p->rho0 * (2.0 * p->r) * (2.0 * p->r) * (2.0 * p->r);
    w->k0 = or_W(0.0, p->h);
    or_grid g;
    or_grid_make(p->h, p->domain_min, p->domain_max, &g);
    uint32_t *perm, *start;
    float *xs;
    sort_points(&g, xf, nf, &perm, &xs, &start);
    build_csr(&g, xs, perm, nf, xs, perm, start, nf, 1, 1, &w->ff);
    w->fb.start = calloc((size_t)(nf + 1), sizeof(int64_t));
    w->fb.idx = malloc(sizeof(uint32_t));
    w->x = malloc(sizeof(double) * 3 * nf);
    for (int64_t i = 0; i < 3 * nf; ++i) w->x[i] = xf[i];
    w->rho = malloc(sizeof(double) * nf); w->alpha = malloc(sizeof(double) * nf); w->Salpha = malloc(sizeof(double) * nf);
    w->psi = NULL;
    density_alpha(w);
    double mu = p->visc * p->rho0;
    int64_t n3 = 3 * nf;
    if (n3 <= 0) return 0;
    double *e = calloc((size_t)n3, sizeof(double)), *col = malloc(sizeof(double) * (size_t)n3);
    for (int64_t c = 0; c < n3; ++c) {
        e[c] = 1.0;
        visc_M(w, mu, e, col);
        for (int64_t r = 0; r < n3; ++r) M[r * n3 + c] = col[r];
        e[c] = 0.0;
    }
    memcpy(rho_out, w->rho, sizeof(double) * nf);
    free(e); free(col);
    free(w->x); free(w->rho); free(w->alpha); free(w->Salpha);
    csr_free(&w->ff); csr_free(&w->fb);
    free(perm); free(start); free(xs);
    return 0;
}

/* CG solve of (I - dt A) v = b alone (for the library-routine pin) */
int or_visc_solve(const or_params *p, const float *xf, int64_t nf, double dt, const double *b, double *x,
                  int32_t *iters, double *resid) {
    world W_, *w = &W_;
    memset(w, 0, sizeof(*w));
    w->p = p; w->nf = nf; w->h = p->h; w->dt = dt;
    w->m = p->rho0 * (2.0 * p->r) * (2.0 * p->r) * (2.0 * p->r);
    w->k0 = or_W(0.0, p->h);
    or_grid g;
    or_grid_make(p->h, p->domain_min, p->domain_max, &g);
    uint32_t *perm, *start;
    float *xs;
    sort_points(&g, xf, nf, &perm, &xs, &start);
    build_csr(&g, xs, perm, nf, xs, perm, start, nf, 1, nf <= 20000, &w->ff);
    w->fb.start = calloc((size_t)(nf + 1), sizeof(int64_t));
    w->fb.idx = malloc(sizeof(uint32_t));
    w->x = malloc(sizeof(double) * 3 * nf);
    for (int64_t i = 0; i < 3 * nf; ++i) w->x[i] = xf[i];
    w->rho = malloc(sizeof(double) * nf); w->alpha = malloc(sizeof(double) * nf); w->Salpha = malloc(sizeof(double) * nf);
    density_alpha(w);
    memcpy(x, b, sizeof(double) * 3 * nf);
    visc_cg(w, p->visc * p->rho0, b, x, iters, resid);
    free(w->x); free(w->rho); free(w->alpha); free(w->Salpha);
    csr_free(&w->ff); csr_free(&w->fb);
    free(perm); free(start); free(xs);
    return 0;
}

/* residual |b - M x| / |b| of a given x, evaluated in FP64 (for checking a
 * GPU solution by its property) */
double or_visc_residual(const or_params *p, const float *xf, const double *rho, int64_t nf, double dt,
                        const double *b, const double *x) {
    world W_, *w = &W_;
    memset(w, 0, sizeof(*w));
    w->p = p; w->nf = nf; w->h = p->h; w->dt = dt;
    w->m = p->rho0 * (2.0 * p->r) * (2.0 * p->r) * (2.0 * p->r);
    or_grid g;
    or_grid_make(p->h, p->domain_min, p->domain_max, &g);
    uint32_t *perm, *start;
    float *xs;
    sort_points(&g, xf, nf, &perm, &xs, &start);
    build_csr(&g, xs, perm, nf, xs, perm, start, nf, 1, 0, &w->ff);
    w->x = malloc(sizeof(double) * 3 * nf);
    for (int64_t i = 0; i < 3 * nf; ++i) w->x[i] = xf[i];
    w->rho = (double *)rho;
    double *Mx = malloc(sizeof(double) * 3 * nf);
    visc_M(w, p->visc * p->rho0, x, Mx);
    double rn = 0.0, bn = 0.0;
    for (int64_t i = 0; i < 3 * nf; ++i) { double r = b[i] - Mx[i]; rn += r * r; bn += b[i] * b[i]; }
    free(Mx); free(w->x);
    csr_free(&w->ff);
    free(perm); free(start); free(xs);
    return bn > 0 ? sqrt(rn / bn) : sqrt(rn);
}

/* density and alpha only (pins on lattices) */
int or_density_alpha(const or_params *p, const float *xf, int64_t nf, const float *xb, int64_t nb,
                     double *rho, double *alpha, double *psi_out) {
    or_in in;
    memset(&in, 0, sizeof(in));
    world W_, *w = &W_;
    memset(w, 0, sizeof(*w));
    w->p = p; w->nf = nf; w->nb = nb; w->h = p->h;
    w->m = p->rho0 * (2.0 * p->r) * (2.0 * p->r) * (2.0 * p->r);
    w->k0 = or_W(0.0, p->h);
    or_grid g;
    or_grid_make(p->h, p->domain_min, p->domain_max, &g);
    uint32_t *pf, *sf, *pb, *sbb;
    float *xsf, *xsb;
    sort_points(&g, xf, nf, &pf, &xsf, &sf);
    sort_points(&g, xb, nb, &pb, &xsb, &sbb);
    int brute = (nf + nb) <= 20000;
    build_csr(&g, xsf, pf, nf, xsf, pf, sf, nf, 1, brute, &w->ff);
    build_csr(&g, xsf, pf, nf, xsb, pb, sbb, nb, 0, brute, &w->fb);
    csr bb;
    build_csr(&g, xsb, pb, nb, xsb, pb, sbb, nb, 1, brute, &bb);
    w->x = malloc(sizeof(double) * 3 * (nf ? nf : 1));
    w->xb = malloc(sizeof(double) * 3 * (nb ? nb : 1));
    for (int64_t i = 0; i < 3 * nf; ++i) w->x[i] = xf[i];
    for (int64_t i = 0; i < 3 * nb; ++i) w->xb[i] = xb[i];
    w->psi = malloc(sizeof(double) * (nb ? nb : 1));
    boundary_psi(p, w->xb, nb, &bb, w->psi);
    w->rho = rho; w->alpha = alpha; w->Salpha = malloc(sizeof(double) * (nf ? nf : 1));
    density_alpha(w);
    if (psi_out) memcpy(psi_out, w->psi, sizeof(double) * nb);
    free(w->x); free(w->xb); free(w->psi); free(w->Salpha);
    csr_free(&w->ff); csr_free(&w->fb); csr_free(&bb);
    free(pf); free(sf); free(xsf); free(pb); free(sbb); free(xsb);
    return 0;
}
