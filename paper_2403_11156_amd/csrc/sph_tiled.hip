// sph_tiled.hip -- cell-row tiles: LDS-staged neighbour build and passes.
//
// A tile is up to kTile consecutive sorted fluid particles of one (cy, cz)
// row of cells, cells cxa..cxb.  Its 27-cell stencil is, per particle set,
// nine contiguous ranges of sorted indices (rows dz, dy = -1..1, cells
// cxa-1..cxb+1), ascending and disjoint; the three ranges of one dz form a
// slab.  A workgroup per tile copies one slab at a time into LDS with
// coalesced loads and every particle of the tile visits the neighbours that
// lie in it, so the neighbour gathers of a pass read LDS instead of the vector
// caches.  The lists of such tiles hold 16-bit slots (slot = range offset +
// position in the range), half the bytes of a sorted index.  Neighbours are
// visited in the order of the untiled kernels (ascending sorted index, fluid
// before boundary), so the sums are the same.  Tiles with a slab of more than
// kSlab particles keep 32-bit sorted indices and gather from global memory.
#include <hip/hip_runtime.h>
#include <algorithm>

#include "sph_device.h"
#include "sph_internal.h"

namespace sph {
namespace {

constexpr int kCapF = kTileCapF;   // LDS list capacity per particle (fluid)
constexpr int kCapB = kTileCapB;   // and boundary

// LDS position of staged particle q: one 16-byte pad after every eight, so
// that the records of particles a cell (about eight particles) apart fall in
// different banks; without it the lanes of a wave, which work on consecutive
// cells, read the same banks.
constexpr int kSlabPad = kSlab + kSlab / 8;
__device__ __forceinline__ int lds(int q) { return q + (q >> 3); }

inline uint32_t tile_blocks(int64_t ntiles) {
    int64_t b = ntiles < 1 ? 1 : ntiles;
    return (uint32_t)((b + 7) & ~int64_t(7));
}

// FP64 sum over a kTile workgroup in a fixed order; valid in thread 0.
__device__ double tile_sum(double v) {
    __shared__ double ws[kTile / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = ws[0];
        for (int w = 1; w < kTile / 64; ++w) r += ws[w];
    }
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- tiles
__global__ void k_row_tile_count(const uint32_t* __restrict__ start_f, Grid g, uint32_t* __restrict__ tilecnt) {
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nrows = (int64_t)g.n[1] * g.n[2], nx = g.n[0];
    if (row >= nrows) return;
    const uint32_t b = start_f[row * nx], e = start_f[row * nx + nx];
    tilecnt[row] = (e - b + kTile - 1) / kTile;
}

// tilerow[t] = the row of tile t
__global__ void k_row_tile_mark(const uint32_t* __restrict__ tileoff, int64_t nrows, uint32_t* __restrict__ tilerow) {
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row >= nrows) return;
    for (uint32_t t = tileoff[row]; t < tileoff[row + 1]; ++t) tilerow[t] = (uint32_t)row;
}

// One thread per tile: its particle range and the nine ranges of its stencil.
__global__ void k_tile_fill(const float4* __restrict__ x, const uint32_t* __restrict__ start_f,
                            const uint32_t* __restrict__ start_b, Grid g, const uint32_t* __restrict__ tileoff,
                            const uint32_t* __restrict__ tilerow, int32_t limit, TileDesc* __restrict__ tiles) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t nx = g.n[0], ny = g.n[1], nz = g.n[2];
    if (t >= (int64_t)tileoff[(int64_t)ny * nz]) return;
    const int64_t row = tilerow[t];
    const int32_t cy = (int32_t)(row % ny), cz = (int32_t)(row / ny);
    const uint32_t e = start_f[row * nx + nx];
    const uint32_t p0 = start_f[row * nx] + (uint32_t)(t - tileoff[row]) * (uint32_t)kTile;
    const uint32_t p1 = min(p0 + (uint32_t)kTile, e);
    // the row's particles are sorted by cx: the first and last bound the tile
    const int32_t cxa = cell_coord(x[p0].x, g.o[0], g.inv, nx);
    const int32_t cxb = cell_coord(x[p1 - 1].x, g.o[0], g.inv, nx);
    TileDesc d;
    d.p0 = (int32_t)p0;
    d.p1 = (int32_t)p1;
    d.pad = 0;
    int32_t fo = 0, bo = 0, ok = 1;
    for (int r = 0; r < 9; ++r) {
        const int32_t z = cz + r / 3 - 1, y = cy + r % 3 - 1;
        uint32_t fb = 0, fe = 0, bb = 0, be = 0;
        if (z >= 0 && z < nz && y >= 0 && y < ny) {
            const int64_t rowp = (int64_t)nx * (y + (int64_t)ny * z);
            const int64_t lo = rowp + (cxa > 0 ? cxa - 1 : 0), hi = rowp + (cxb < nx - 1 ? cxb + 1 : nx - 1);
            fb = start_f[lo];
            fe = start_f[hi + 1];
            bb = start_b[lo];
            be = start_b[hi + 1];
        }
        d.fb[r] = (int32_t)fb;
        d.foff[r] = fo;
        fo += (int32_t)(fe - fb);
        d.bb[r] = (int32_t)bb;
        d.boff[r] = bo;
        bo += (int32_t)(be - bb);
        if (r % 3 == 2) {
            if (fo - d.foff[r - 2] > limit || bo - d.boff[r - 2] > limit) ok = 0;
        }
    }
    d.foff[9] = fo;
    d.boff[9] = bo;
    d.ok = ok;
    tiles[t] = d;
}

// Slab s of a set: its three ranges laid end to end, position q of the slab
// holding sorted index src(q).
struct SlabMap {
    int32_t n, l1, l2, b0, b1, b2;
};

__device__ __forceinline__ SlabMap slab_map(const int32_t* first, const int32_t* off, int s) {
    const int32_t o0 = off[3 * s];
    SlabMap m;
    m.l1 = off[3 * s + 1] - o0;
    m.l2 = off[3 * s + 2] - o0;
    m.n = off[3 * s + 3] - o0;
    m.b0 = first[3 * s];
    m.b1 = first[3 * s + 1] - m.l1;
    m.b2 = first[3 * s + 2] - m.l2;
    return m;
}

__device__ __forceinline__ int32_t slab_src(SlabMap m, int32_t q) {
    return (q < m.l1 ? m.b0 : (q < m.l2 ? m.b1 : m.b2)) + q;
}

constexpr int kStageIters = (kSlab + kTile - 1) / kTile;

// Copy slab m of one, two or three arrays into LDS: the workgroup's loads
// (positions past the slab re-read its first element, a valid index whenever
// the slab is not empty) are all issued before the first LDS store, so the
// copy costs one memory latency.  An empty slab loads nothing (uniform).
#define SPH_STAGE_LOADS(u)                                                      \
    const int32_t q##u = (int32_t)threadIdx.x + (u) * kTile;                    \
    const int32_t j##u = slab_src(m, q##u < m.n ? q##u : 0);
#define SPH_STAGE_ALL(X) X(0) X(1) X(2) X(3) X(4)
static_assert(kStageIters == 5, "SPH_STAGE_ALL unrolls five iterations");

template <class T0>
__device__ __forceinline__ void stage(SlabMap m, T0* d0, const T0* __restrict__ a0) {
    if (m.n == 0) return;
    SPH_STAGE_ALL(SPH_STAGE_LOADS)
#define L_(u) const T0 v0_##u = a0[j##u];
    SPH_STAGE_ALL(L_)
#undef L_
#define S_(u) if (q##u < m.n) d0[lds(q##u)] = v0_##u;
    SPH_STAGE_ALL(S_)
#undef S_
}

template <class T0, class T1>
__device__ __forceinline__ void stage(SlabMap m, T0* d0, const T0* __restrict__ a0, T1* d1,
                                      const T1* __restrict__ a1) {
    if (m.n == 0) return;
    SPH_STAGE_ALL(SPH_STAGE_LOADS)
#define L_(u) const T0 v0_##u = a0[j##u]; const T1 v1_##u = a1[j##u];
    SPH_STAGE_ALL(L_)
#undef L_
#define S_(u) if (q##u < m.n) { d0[lds(q##u)] = v0_##u; d1[lds(q##u)] = v1_##u; }
    SPH_STAGE_ALL(S_)
#undef S_
}

template <class T0, class T1, class T2>
__device__ __forceinline__ void stage(SlabMap m, T0* d0, const T0* __restrict__ a0, T1* d1,
                                      const T1* __restrict__ a1, T2* d2, const T2* __restrict__ a2) {
    if (m.n == 0) return;
    SPH_STAGE_ALL(SPH_STAGE_LOADS)
#define L_(u) const T0 v0_##u = a0[j##u]; const T1 v1_##u = a1[j##u]; const T2 v2_##u = a2[j##u];
    SPH_STAGE_ALL(L_)
#undef L_
#define S_(u) if (q##u < m.n) { d0[lds(q##u)] = v0_##u; d1[lds(q##u)] = v1_##u; d2[lds(q##u)] = v2_##u; }
    SPH_STAGE_ALL(S_)
#undef S_
}
#undef SPH_STAGE_ALL
#undef SPH_STAGE_LOADS

// Visit the list entries k.. of one particle whose slots lie below `end`
// (the slots ascend, so they form a prefix), as LDS positions lds(slot - base).
// List loads go four at a time ahead of the work, as in for_each_nbr.
template <class F>
__device__ __forceinline__ void slab_slots(const uint16_t*& p, int64_t nf, uint32_t n, uint32_t& k, uint32_t end,
                                           uint32_t base, F&& f) {
    while (k + 4 <= n) {
        const uint32_t s0 = p[0], s1 = p[nf], s2 = p[2 * nf], s3 = p[3 * nf];
        if (s3 < end) {
            f(lds(s0 - base));
            f(lds(s1 - base));
            f(lds(s2 - base));
            f(lds(s3 - base));
            k += 4;
            p += 4 * nf;
            continue;
        }
        if (s0 < end) {
            f(lds(s0 - base));
            ++k;
            p += nf;
            if (s1 < end) {
                f(lds(s1 - base));
                ++k;
                p += nf;
                if (s2 < end) {
                    f(lds(s2 - base));
                    ++k;
                    p += nf;
                }
            }
        }
        return;
    }
    while (k < n) {
        const uint32_t s0 = *p;
        if (s0 >= end) return;
        f(lds(s0 - base));
        ++k;
        p += nf;
    }
}

// One set's neighbours of the tile particle i, slab by slab: stage_fn(map)
// copies the slab into LDS, fn(position) does one neighbour.  Every thread of the
// workgroup calls this (the barriers); threads without a particle pass mine =
// false.
template <class Stage, class Fn>
__device__ __forceinline__ void sweep(const uint16_t* __restrict__ list, const uint32_t* __restrict__ cnt, int64_t nf,
                                      int64_t i, bool mine, const int32_t* first, const int32_t* off,
                                      Stage&& stage_fn, Fn&& fn) {
    if (off[9] == 0) return;   // no particle of this set near the tile (uniform)
    const uint32_t n = mine ? cnt[i] : 0u;
    uint32_t k = 0;
    const uint16_t* p = list + (mine ? i : 0);
    for (int s = 0; s < 3; ++s) {
        if (off[3 * s + 3] == off[3 * s]) continue;   // empty slab (uniform)
        stage_fn(slab_map(first, off, s));
        __syncthreads();
        slab_slots(p, nf, n, k, (uint32_t)off[3 * s + 3], (uint32_t)off[3 * s], fn);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- neighbour build
__global__ void __launch_bounds__(kTile) k_nbr_build_tiled(
    const TileDesc* __restrict__ tiles, const uint32_t* __restrict__ ntiles_dev, const float4* __restrict__ x,
    int64_t nf, const float4* __restrict__ xb, const uint32_t* __restrict__ start_f,
    const uint32_t* __restrict__ start_b, Grid g, uint16_t* __restrict__ l16, uint32_t* __restrict__ l32,
    uint32_t* __restrict__ ncnt, int32_t capf, uint16_t* __restrict__ b16, uint32_t* __restrict__ b32,
    uint32_t* __restrict__ bcnt, int32_t capb, uint32_t* flags, unsigned long long* __restrict__ stats) {
    __shared__ float4 sx[kSlabPad];
    __shared__ float4 sb[kSlabPad];
    __shared__ uint16_t lf[kCapF * kTile];
    __shared__ uint16_t lb[kCapB * kTile];
    const uint32_t t = logical_block();
    uint32_t total = 0xffffffffu, fl = 0;
    bool mine = false, over = false;
    if (t < *ntiles_dev) {
        const TileDesc& d = tiles[t];
        const int64_t i = d.p0 + (int64_t)threadIdx.x;
        mine = i < d.p1;
        over = d.ok == 0;
        uint32_t nfc = 0, nbc = 0;
        float4 xi = make_float4(0.f, 0.f, 0.f, 0.f);
        int32_t cx = 0, cy = 0, cz = 0;
        if (mine) {
            xi = x[i];
            cx = cell_coord(xi.x, g.o[0], g.inv, g.n[0]);
            cy = cell_coord(xi.y, g.o[1], g.inv, g.n[1]);
            cz = cell_coord(xi.z, g.o[2], g.inv, g.n[2]);
        }
        const int32_t x0 = cx > 0 ? cx - 1 : 0, x1 = cx < g.n[0] - 1 ? cx + 1 : g.n[0] - 1;
        if (d.ok) {
            for (int s = 0; s < 3; ++s) {
                if (d.foff[3 * s + 3] == d.foff[3 * s] && d.boff[3 * s + 3] == d.boff[3 * s]) continue;
                stage(slab_map(d.fb, d.foff, s), sx, x);
                stage(slab_map(d.bb, d.boff, s), sb, xb);
                __syncthreads();
                const int32_t z = cz + s - 1;
                if (mine && z >= 0 && z < g.n[2]) {
                    for (int32_t dy = -1; dy <= 1; ++dy) {
                        const int32_t y = cy + dy;
                        if (y < 0 || y >= g.n[1]) continue;
                        const int r = 3 * s + dy + 1;
                        const int64_t row = (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z);
                        {
                            // candidate j: slot foff[r] + (j - fb[r]), LDS index slot - foff[3s]
                            const int32_t slot0 = d.foff[r] - d.fb[r], lds0 = slot0 - d.foff[3 * s];
                            const uint32_t b = start_f[row + x0], e = start_f[row + x1 + 1];
                            auto take = [&](uint32_t j, float4 pj) {
                                if ((int64_t)j != i && dist2_exact(xi, pj) < g.h2) {
                                    if (nfc < (uint32_t)capf)
                                        lf[nfc * kTile + threadIdx.x] = (uint16_t)(slot0 + (int32_t)j);
                                    ++nfc;
                                }
                            };
                            uint32_t j = b;
                            for (; j + 4 <= e; j += 4) {
                                const int32_t q = lds0 + (int32_t)j;
                                const float4 q0 = sx[lds(q)], q1 = sx[lds(q + 1)], q2 = sx[lds(q + 2)],
                                             q3 = sx[lds(q + 3)];
                                take(j, q0);
                                take(j + 1, q1);
                                take(j + 2, q2);
                                take(j + 3, q3);
                            }
                            for (; j < e; ++j) take(j, sx[lds(lds0 + (int32_t)j)]);
                        }
                        {
                            const int32_t slot0 = d.boff[r] - d.bb[r], lds0 = slot0 - d.boff[3 * s];
                            const uint32_t b = start_b[row + x0], e = start_b[row + x1 + 1];
                            for (uint32_t k = b; k < e; ++k) {
                                if (dist2_exact(xi, sb[lds(lds0 + (int32_t)k)]) < g.h2) {
                                    if (nbc < (uint32_t)capb)
                                        lb[nbc * kTile + threadIdx.x] = (uint16_t)(slot0 + (int32_t)k);
                                    ++nbc;
                                }
                            }
                        }
                    }
                }
                __syncthreads();
            }
            if (mine) {
                // neighbour-major flush: lanes of a wave write adjacent entries
                const uint32_t nfs = min(nfc, (uint32_t)capf), nbs = min(nbc, (uint32_t)capb);
                for (uint32_t k = 0; k < nfs; ++k) l16[(int64_t)k * nf + i] = lf[k * kTile + threadIdx.x];
                for (uint32_t k = 0; k < nbs; ++k) b16[(int64_t)k * nf + i] = lb[k * kTile + threadIdx.x];
            }
        } else if (mine) {
            // over-full tile: 32-bit sorted indices from a global-memory search
            uint4 fbuf = make_uint4(0u, 0u, 0u, 0u), bbuf = make_uint4(0u, 0u, 0u, 0u);
            for (int32_t dz = -1; dz <= 1; ++dz) {
                const int32_t z = cz + dz;
                if (z < 0 || z >= g.n[2]) continue;
                for (int32_t dy = -1; dy <= 1; ++dy) {
                    const int32_t y = cy + dy;
                    if (y < 0 || y >= g.n[1]) continue;
                    const int64_t row = (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z);
                    scan_candidates(x, start_f[row + x0], start_f[row + x1 + 1], xi, i, i, g.h2, l32, nf, capf, nfc,
                                    fbuf);
                    scan_candidates(xb, start_b[row + x0], start_b[row + x1 + 1], xi, i, -1, g.h2, b32, nf, capb,
                                    nbc, bbuf);
                }
            }
            list_flush(l32, nf, i, capf, nfc, fbuf);
            list_flush(b32, nf, i, capb, nbc, bbuf);
        }
        if (mine) {
            ncnt[i] = min(nfc, (uint32_t)capf);
            bcnt[i] = min(nbc, (uint32_t)capb);
            if (nfc > (uint32_t)capf || nbc > (uint32_t)capb) atomicOr(flags, 1u);
            total = nfc + nbc;
            fl = nfc;
        }
    }
    // neighbour statistics of this workgroup (kNStats fields)
    uint32_t mn = total, mx = mine ? total : 0u;
    unsigned long long sm = mine ? total : 0ull, sf = fl, so = (mine && over) ? total : 0ull;
    for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, (uint32_t)__shfl_down((int)mn, off, 64));
        mx = max(mx, (uint32_t)__shfl_down((int)mx, off, 64));
        sm += __shfl_down(sm, off, 64);
        sf += __shfl_down(sf, off, 64);
        so += __shfl_down(so, off, 64);
    }
    __shared__ unsigned long long ws[kTile / 64][5];
    if ((threadIdx.x & 63) == 0) {
        ws[threadIdx.x >> 6][0] = mn;
        ws[threadIdx.x >> 6][1] = mx;
        ws[threadIdx.x >> 6][2] = sm;
        ws[threadIdx.x >> 6][3] = sf;
        ws[threadIdx.x >> 6][4] = so;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = ws[0][0], b = ws[0][1], c = ws[0][2], e = ws[0][3], o4 = ws[0][4];
        for (int w = 1; w < kTile / 64; ++w) {
            a = min(a, ws[w][0]);
            b = max(b, ws[w][1]);
            c += ws[w][2];
            e += ws[w][3];
            o4 += ws[w][4];
        }
        unsigned long long* o = stats + (size_t)kNStats * blockIdx.x;
        o[0] = a;
        o[1] = b;
        o[2] = c;
        o[3] = e;
        o[4] = o4;
        o[5] = over ? 1ull : 0ull;
    }
}

// ---------------------------------------------------------------- passes
// Each pass: one workgroup per tile; in an ok tile the fluid neighbours are
// swept slab by slab from LDS, then the boundary neighbours the same way; an
// over-full tile gathers through its 32-bit lists as the untiled kernels do.
// The per-neighbour arithmetic is written once per pass as a lambda taking
// the neighbour's staged values.

__global__ void __launch_bounds__(kTile) k_density_alpha_t(Lists L, int64_t nf, float4* __restrict__ x,
                                                           const float4* __restrict__ v,
                                                           const float4* __restrict__ xb, Kern kc,
                                                           float* __restrict__ rho, float* __restrict__ alpha,
                                                           float4* __restrict__ v_in, float* __restrict__ Kv,
                                                           float* __restrict__ kappa, float warm_factor) {
    __shared__ float4 s0[kSlabPad];
    const uint32_t t = logical_block();
    if (t >= L.ntiles) return;
    const TileDesc& d = L.tiles[t];
    const int64_t i = d.p0 + (int64_t)threadIdx.x;
    const bool mine = i < d.p1;
    const float4 xi = mine ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float r = kc.m * kc.k;
    float gx = 0.f, gy = 0.f, gz = 0.f, sq = 0.f;
    auto fluid = [&](float4 xj) {
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        r += kc.m * kernel_W(r2, kc);
        const float F = kc.m * grad_factor(r2, kc);
        const float ax = F * dx, ay = F * dy, az = F * dz;
        gx += ax; gy += ay; gz += az;
        sq += ax * ax + ay * ay + az * az;
    };
    auto bound = [&](float4 xk) {
        const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        r += xk.w * kernel_W(r2, kc);
        const float F = xk.w * grad_factor(r2, kc);
        gx += F * dx; gy += F * dy; gz += F * dz;
    };
    if (d.ok) {
        sweep(L.l16, L.ncnt, nf, i, mine, d.fb, d.foff, [&](SlabMap m) { stage(m, s0, (const float4*)x); },
              [&](uint32_t q) { fluid(s0[q]); });
        sweep(L.b16, L.bcnt, nf, i, mine, d.bb, d.boff, [&](SlabMap m) { stage(m, s0, xb); },
              [&](uint32_t q) { bound(s0[q]); });
    } else if (mine) {
        for_each_nbr(L.l32, nf, i, L.ncnt[i], [&](uint32_t j) { fluid(x[j]); });
        for_each_nbr(L.b32, nf, i, L.bcnt[i], [&](uint32_t k) { bound(xb[k]); });
    }
    if (!mine) return;
    const float D = gx * gx + gy * gy + gz * gz + sq;
    rho[i] = r;
    alpha[i] = D > 1e-6f ? r / D : 0.0f;
    v_in[i] = v[i];
    const float k0 = warm_factor * Kv[i];
    kappa[i] = k0;
    Kv[i] = 0.0f;
    x[i].w = k0 / r;
}

__global__ void __launch_bounds__(kTile) k_pressure_update_t(Lists L, int64_t nf, const float4* __restrict__ x,
                                                             float4* __restrict__ v,
                                                             const float* __restrict__ kappa,
                                                             float* __restrict__ Kacc,
                                                             float* __restrict__ kappa_last,
                                                             const float4* __restrict__ xb, Kern kc, float dt,
                                                             const int32_t* __restrict__ go) {
    __shared__ float4 s0[kSlabPad];
    if (go != nullptr && *go == 0) return;
    const uint32_t t = logical_block();
    if (t >= L.ntiles) return;
    const TileDesc& d = L.tiles[t];
    const int64_t i = d.p0 + (int64_t)threadIdx.x;
    const bool mine = i < d.p1;
    const float4 xi = mine ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float kri = xi.w;
    float ax = 0.f, ay = 0.f, az = 0.f;
    auto fluid = [&](float4 xj) {
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float c = (kri + xj.w) * grad_factor(r2, kc);
        ax += c * dx; ay += c * dy; az += c * dz;
    };
    auto bound = [&](float4 xk) {
        const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float c = xk.w * kri * grad_factor(r2, kc);
        ax += c * dx; ay += c * dy; az += c * dz;
    };
    if (d.ok) {
        sweep(L.l16, L.ncnt, nf, i, mine, d.fb, d.foff, [&](SlabMap m) { stage(m, s0, x); },
              [&](uint32_t q) { fluid(s0[q]); });
        ax *= kc.m; ay *= kc.m; az *= kc.m;
        sweep(L.b16, L.bcnt, nf, i, mine, d.bb, d.boff, [&](SlabMap m) { stage(m, s0, xb); },
              [&](uint32_t q) { bound(s0[q]); });
    } else if (mine) {
        for_each_nbr(L.l32, nf, i, L.ncnt[i], [&](uint32_t j) { fluid(x[j]); });
        ax *= kc.m; ay *= kc.m; az *= kc.m;
        for_each_nbr(L.b32, nf, i, L.bcnt[i], [&](uint32_t k) { bound(xb[k]); });
    }
    if (!mine) return;
    float4 vi = v[i];
    vi.x -= dt * ax; vi.y -= dt * ay; vi.z -= dt * az;
    v[i] = vi;
    const float ki = kappa[i];
    Kacc[i] += ki;
    if (kappa_last) kappa_last[i] = ki;
}

// Density change rate of the current velocities at the tile particle i (fluid
// sum times m, then the boundary terms), handed to fin: the shared core of
// the solver's predict pass and of the warm-start features.
template <class Fin>
__device__ __forceinline__ void divergence_tile(const Lists& L, int64_t nf, const TileDesc& d, int64_t i, bool mine,
                                                const float4* __restrict__ x, const float4* __restrict__ v,
                                                const float4* __restrict__ xb, const float4* __restrict__ vb,
                                                const Kern& kc, float4* s0, float4* s1, Fin&& fin) {
    const float4 xi = mine ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 vi = mine ? v[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float dd = 0.f;
    auto fluid = [&](float4 xj, float4 vj) {
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        dd += grad_factor(r2, kc) * ((vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz);
    };
    auto bound = [&](float4 xk, float4 vk) {
        const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        dd += xk.w * grad_factor(r2, kc) * ((vi.x - vk.x) * dx + (vi.y - vk.y) * dy + (vi.z - vk.z) * dz);
    };
    if (d.ok) {
        sweep(L.l16, L.ncnt, nf, i, mine, d.fb, d.foff, [&](SlabMap m) { stage(m, s0, x, s1, v); },
              [&](uint32_t q) { fluid(s0[q], s1[q]); });
        dd *= kc.m;
        sweep(L.b16, L.bcnt, nf, i, mine, d.bb, d.boff, [&](SlabMap m) { stage(m, s0, xb, s1, vb); },
              [&](uint32_t q) { bound(s0[q], s1[q]); });
    } else if (mine) {
        for_each_nbr(L.l32, nf, i, L.ncnt[i], [&](uint32_t j) { fluid(x[j], v[j]); });
        dd *= kc.m;
        for_each_nbr(L.b32, nf, i, L.bcnt[i], [&](uint32_t k) { bound(xb[k], vb[k]); });
    }
    fin(dd);
}

template <int MODE>
__global__ void __launch_bounds__(kTile) k_predict_t(Lists L, int64_t nf, float4* __restrict__ x,
                                                     const float4* __restrict__ v, const float* __restrict__ rho,
                                                     const float* __restrict__ alpha, float* __restrict__ kappa,
                                                     const float4* __restrict__ xb, const float4* __restrict__ vb,
                                                     Kern kc, float dt, double* __restrict__ partials,
                                                     const int32_t* __restrict__ go, float* __restrict__ dout) {
    __shared__ float4 s0[kSlabPad];
    __shared__ float4 s1[kSlabPad];
    if (go != nullptr && *go == 0) return;
    const uint32_t t = logical_block();
    double e = 0.0;
    if (t < L.ntiles) {
        const TileDesc& d = L.tiles[t];
        const int64_t i = d.p0 + (int64_t)threadIdx.x;
        const bool mine = i < d.p1;
        divergence_tile(L, nf, d, i, mine, x, v, xb, vb, kc, s0, s1, [&](float dd) {
            if (!mine) return;
            const float ri = rho[i];
            float kap;
            if (MODE == 0) {
                if (dout) dout[i] = dd;
                const float ep = fmaxf(dd, 0.0f);
                kap = ep * alpha[i] / dt;
                e = (double)ep;
            } else {
                const float dev = (ri - kc.rho0) + dt * dd;
                const float ep = fmaxf(dev, 0.0f);
                kap = ep * alpha[i] / (dt * dt);
                e = (double)ep;
            }
            kappa[i] = kap;
            x[i].w = kap / ri;
        });
    }
    const double bs = tile_sum(e);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

template <int MODEL>
__global__ void __launch_bounds__(kTile) k_nonpressure_t(Lists L, int64_t nf, float4* __restrict__ x,
                                                         const float4* __restrict__ v, float4* __restrict__ vout,
                                                         const float* __restrict__ rho, Kern kc, float dt, float gx,
                                                         float gy, float gz, float visc, float* __restrict__ K,
                                                         float* __restrict__ kappa, float warm_factor,
                                                         bool setup_warm) {
    __shared__ float4 s0[MODEL != 0 ? kSlabPad : 1];
    __shared__ float4 s1[MODEL != 0 ? kSlabPad : 1];
    __shared__ float s2[MODEL != 0 ? kSlabPad : 1];
    const uint32_t t = logical_block();
    if (t >= L.ntiles) return;
    const TileDesc& d = L.tiles[t];
    const int64_t i = d.p0 + (int64_t)threadIdx.x;
    const bool mine = i < d.p1;
    const float4 xi = mine ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 vi = mine ? v[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float ax = 0.f, ay = 0.f, az = 0.f;
    if (MODEL == 1 || MODEL == 2) {
        const float eps2 = 0.01f * kc.h * kc.h;
        auto fluid = [&](float4 xj, float4 vj, float rj) {
            const float mj = kc.m / rj;
            const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (MODEL == 1) {
                const float c = mj * kernel_W(r2, kc);
                ax += c * (vj.x - vi.x); ay += c * (vj.y - vi.y); az += c * (vj.z - vi.z);
            } else {
                const float vx = (vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz;
                const float c = mj * vx / (r2 + eps2) * grad_factor(r2, kc);
                ax += c * dx; ay += c * dy; az += c * dz;
            }
        };
        if (d.ok)
            sweep(L.l16, L.ncnt, nf, i, mine, d.fb, d.foff,
                  [&](SlabMap m) { stage(m, s0, (const float4*)x, s1, v, s2, rho); },
                  [&](uint32_t q) { fluid(s0[q], s1[q], s2[q]); });
        else if (mine)
            for_each_nbr(L.l32, nf, i, L.ncnt[i], [&](uint32_t j) { fluid(x[j], v[j], rho[j]); });
    }
    if (!mine) return;
    float s = 0.f;
    if (MODEL == 1) s = visc;
    if (MODEL == 2) s = dt * visc * 2.0f * (3 + 2);
    float4 o;
    o.x = vi.x + dt * gx + s * ax;
    o.y = vi.y + dt * gy + s * ay;
    o.z = vi.z + dt * gz + s * az;
    o.w = 0.f;
    vout[i] = o;
    if (setup_warm) {
        const float k0 = warm_factor * K[i];
        kappa[i] = k0;
        K[i] = 0.0f;
        x[i].w = k0 / rho[i];
    }
}

// Reaction on the rigid bodies: the untiled kernel's arithmetic over the
// tile's particles, the boundary neighbour recovered from its slot through the
// tile's ranges.  No staging (the boundary lists of most tiles are empty).
__global__ void __launch_bounds__(kTile) k_rigid_force_t(Lists L, int64_t nf, const float4* __restrict__ x,
                                                         const float* __restrict__ rho, const float* __restrict__ K,
                                                         const float* __restrict__ Kv,
                                                         const float4* __restrict__ xb,
                                                         const float4* __restrict__ vb, Kern kc, int32_t nbody,
                                                         const double* __restrict__ com,
                                                         double* __restrict__ partials) {
    const uint32_t t = logical_block();
    uint32_t nbk = 0;
    bool ok = true;
    int64_t i = 0;
    float4 xi = make_float4(0.f, 0.f, 0.f, 0.f);
    float base = 0.f;
    const TileDesc* d = nullptr;
    if (t < L.ntiles) {
        d = &L.tiles[t];
        ok = d->ok != 0;
        i = d->p0 + (int64_t)threadIdx.x;
        if (i < d->p1) {
            nbk = L.bcnt[i];
            if (nbk) {
                xi = x[i];
                base = kc.m * (K[i] + Kv[i]) / rho[i];
            }
        }
    }
    for (int32_t b = 0; b < nbody; ++b) {
        double f[3] = {0.0, 0.0, 0.0}, tq[3] = {0.0, 0.0, 0.0};
        for (uint32_t k = 0; k < nbk; ++k) {
            uint32_t kk;
            if (ok) {
                const int32_t s = L.b16[(int64_t)k * nf + i];
                int r = 0;
                while (r < 8 && s >= d->boff[r + 1]) ++r;
                kk = (uint32_t)(d->bb[r] + (s - d->boff[r]));
            } else {
                kk = L.b32[list_index(nf, i, k)];
            }
            const float4 vk = vb[kk];
            if ((int32_t)vk.w != b) continue;
            const float4 xk = xb[kk];
            const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float c = base * xk.w * grad_factor(r2, kc);
            const double Fx = (double)(c * dx), Fy = (double)(c * dy), Fz = (double)(c * dz);
            const double rx = (double)xk.x - com[3 * b], ry = (double)xk.y - com[3 * b + 1],
                         rz = (double)xk.z - com[3 * b + 2];
            f[0] += Fx; f[1] += Fy; f[2] += Fz;
            tq[0] += ry * Fz - rz * Fy;
            tq[1] += rz * Fx - rx * Fz;
            tq[2] += rx * Fy - ry * Fx;
        }
        for (int c = 0; c < 3; ++c) {
            const double s0 = tile_sum(f[c]);
            const double s1 = tile_sum(tq[c]);
            if (threadIdx.x == 0) {
                partials[((size_t)blockIdx.x * nbody + b) * 6 + c] = s0;
                partials[((size_t)blockIdx.x * nbody + b) * 6 + 3 + c] = s1;
            }
        }
    }
}

__global__ void __launch_bounds__(kTile) k_visc_matvec_t(Lists L, int64_t nf, const float4* __restrict__ x,
                                                         const float* __restrict__ rho, const float4* __restrict__ p,
                                                         float4* __restrict__ Mp, Kern kc, float dt, float mu) {
    __shared__ float4 s0[kSlabPad];
    __shared__ float4 s1[kSlabPad];
    __shared__ float s2[kSlabPad];
    const uint32_t t = logical_block();
    if (t >= L.ntiles) return;
    const TileDesc& d = L.tiles[t];
    const int64_t i = d.p0 + (int64_t)threadIdx.x;
    const bool mine = i < d.p1;
    const float4 xi = mine ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 pi = mine ? p[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float eps2 = 0.01f * kc.h * kc.h;
    float ax = 0.f, ay = 0.f, az = 0.f;
    auto fluid = [&](float4 xj, float4 pj, float rj) {
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float xv = (pi.x - pj.x) * dx + (pi.y - pj.y) * dy + (pi.z - pj.z) * dz;
        const float c = xv / (rj * (r2 + eps2)) * grad_factor(r2, kc);
        ax += c * dx; ay += c * dy; az += c * dz;
    };
    if (d.ok)
        sweep(L.l16, L.ncnt, nf, i, mine, d.fb, d.foff, [&](SlabMap m) { stage(m, s0, x, s1, p, s2, rho); },
              [&](uint32_t q) { fluid(s0[q], s1[q], s2[q]); });
    else if (mine)
        for_each_nbr(L.l32, nf, i, L.ncnt[i], [&](uint32_t j) { fluid(x[j], p[j], rho[j]); });
    if (!mine) return;
    const float s = dt * 10.0f * mu * kc.m / rho[i];
    float4 o;
    o.x = pi.x - s * ax; o.y = pi.y - s * ay; o.z = pi.z - s * az; o.w = 0.f;
    Mp[i] = o;
}

__global__ void __launch_bounds__(kTile) k_visc_precond_t(Lists L, int64_t nf, const float4* __restrict__ x,
                                                          const float* __restrict__ rho, Kern kc, float dt, float mu,
                                                          float* __restrict__ Pinv) {
    __shared__ float4 s0[kSlabPad];
    __shared__ float s2[kSlabPad];
    const uint32_t t = logical_block();
    if (t >= L.ntiles) return;
    const TileDesc& d = L.tiles[t];
    const int64_t i = d.p0 + (int64_t)threadIdx.x;
    const bool mine = i < d.p1;
    const float4 xi = mine ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float eps2 = 0.01f * kc.h * kc.h;
    float b00 = 0.f, b01 = 0.f, b02 = 0.f, b11 = 0.f, b12 = 0.f, b22 = 0.f;
    auto fluid = [&](float4 xj, float rj) {
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float c = grad_factor(r2, kc) / (rj * (r2 + eps2));
        b00 += c * dx * dx; b01 += c * dx * dy; b02 += c * dx * dz;
        b11 += c * dy * dy; b12 += c * dy * dz; b22 += c * dz * dz;
    };
    if (d.ok)
        sweep(L.l16, L.ncnt, nf, i, mine, d.fb, d.foff, [&](SlabMap m) { stage(m, s0, x, s2, rho); },
              [&](uint32_t q) { fluid(s0[q], s2[q]); });
    else if (mine)
        for_each_nbr(L.l32, nf, i, L.ncnt[i], [&](uint32_t j) { fluid(x[j], rho[j]); });
    if (!mine) return;
    const float s = -dt * 10.0f * mu * kc.m / rho[i];
    const double a = 1.0 + (double)(s * b00), bq = (double)(s * b01), cq = (double)(s * b02);
    const double e = 1.0 + (double)(s * b11), f = (double)(s * b12), k2 = 1.0 + (double)(s * b22);
    const double A = e * k2 - f * f, B = -(bq * k2 - f * cq), C = bq * f - e * cq;
    const double det = a * A + bq * B + cq * C;
    const double id = 1.0 / det;
    float* o = Pinv + 9 * i;
    o[0] = (float)(A * id);
    o[1] = (float)(-(bq * k2 - cq * f) * id);
    o[2] = (float)((bq * f - cq * e) * id);
    o[3] = (float)(B * id);
    o[4] = (float)((a * k2 - cq * cq) * id);
    o[5] = (float)(-(a * f - cq * bq) * id);
    o[6] = (float)(C * id);
    o[7] = (float)(-(a * f - bq * cq) * id);
    o[8] = (float)((a * e - bq * bq) * id);
}

}  // namespace

// ================================================================ launchers
int64_t max_tiles(int64_t nf, int64_t nrows) { return nf / kTile + nrows + 1; }
uint32_t tile_partials(int64_t ntiles) { return tile_blocks(ntiles); }

hipError_t launch_tiles_build(const float4* x, const uint32_t* start_f, const uint32_t* start_b, Grid g,
                              int32_t slab_limit, uint32_t* tilecnt, uint32_t* tileoff, uint32_t* tilerow,
                              int64_t max_t, uint32_t* scan_part, TileDesc* tiles, hipStream_t s) {
    if (slab_limit < 0 || slab_limit > kSlab) return hipErrorInvalidValue;
    const int64_t nrows = (int64_t)g.n[1] * g.n[2];
    const uint32_t blocks = (uint32_t)((nrows + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_row_tile_count, dim3(blocks), dim3(kBlock), 0, s, start_f, g, tilecnt);
    hipError_t e = launch_exclusive_scan(tilecnt, nrows, tileoff, scan_part, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_tile_mark, dim3(blocks), dim3(kBlock), 0, s, tileoff, nrows, tilerow);
    const uint32_t tb = (uint32_t)std::max<int64_t>((max_t + kBlock - 1) / kBlock, 1);
    hipLaunchKernelGGL(k_tile_fill, dim3(tb), dim3(kBlock), 0, s, x, start_f, start_b, g, tileoff, tilerow,
                       slab_limit, tiles);
    return hipGetLastError();
}

hipError_t launch_nbr_build_tiled(const TileDesc* tiles, const uint32_t* ntiles_dev, int64_t max_t, const float4* x,
                                  int64_t nf, const float4* xb, const uint32_t* start_f, const uint32_t* start_b,
                                  Grid g, uint16_t* l16, uint32_t* l32, uint32_t* ncnt, int32_t capf, uint16_t* b16,
                                  uint32_t* b32, uint32_t* bcnt, int32_t capb, uint32_t* flags,
                                  unsigned long long* partials, HostStatus* host, hipStream_t s) {
    if (capf > kCapF || capb > kCapB) return hipErrorInvalidValue;
    const uint32_t nblk = tile_blocks(max_t);
    hipLaunchKernelGGL(k_nbr_build_tiled, dim3(nblk), dim3(kTile), 0, s, tiles, ntiles_dev, x, nf, xb, start_f,
                       start_b, g, l16, l32, ncnt, capf, b16, b32, bcnt, capb, flags, partials);
    hipLaunchKernelGGL(k_finish_nstats, dim3(1), dim3(kBlock), 0, s, partials, (int)nblk, (const uint32_t*)flags,
                       ntiles_dev, host);
    return hipGetLastError();
}

#define TLAUNCH(kern, ...)                                                                        \
    do {                                                                                          \
        if (L.ntiles <= 0) return hipSuccess;                                                     \
        hipLaunchKernelGGL(kern, dim3(tile_blocks(L.ntiles)), dim3(kTile), 0, s, L, __VA_ARGS__); \
        return hipGetLastError();                                                                 \
    } while (0)

hipError_t launch_density_alpha_t(const Lists& L, int64_t nf, float4* x, const float4* v, const float4* xb, Kern kc,
                                  float* rho, float* alpha, float4* v_in, float* Kv, float* kappa, float warm_factor,
                                  hipStream_t s) {
    TLAUNCH(k_density_alpha_t, nf, x, v, xb, kc, rho, alpha, v_in, Kv, kappa, warm_factor);
}

hipError_t launch_pressure_update_t(const Lists& L, int64_t nf, const float4* x, float4* v, const float* kappa,
                                    float* Kacc, float* kappa_last, const float4* xb, Kern kc, float dt,
                                    const int32_t* go, hipStream_t s) {
    TLAUNCH(k_pressure_update_t, nf, x, v, kappa, Kacc, kappa_last, xb, kc, dt, go);
}

hipError_t launch_predict_t(int mode, const Lists& L, int64_t nf, float4* x, const float4* v, const float* rho,
                            const float* alpha, float* kappa, const float4* xb, const float4* vb, Kern kc, float dt,
                            double* partials, SolveCtl* ctl, bool first, float* dout, int* nparts, hipStream_t s) {
    const uint32_t nblk = tile_blocks(L.ntiles);
    *nparts = L.ntiles > 0 ? (int)nblk : 0;
    if (L.ntiles <= 0) return hipSuccess;
    const int32_t* go = first ? nullptr : &ctl->go;
    if (mode == 0)
        hipLaunchKernelGGL(k_predict_t<0>, dim3(nblk), dim3(kTile), 0, s, L, nf, x, v, rho, alpha, kappa, xb, vb, kc,
                           dt, partials, go, dout);
    else
        hipLaunchKernelGGL(k_predict_t<1>, dim3(nblk), dim3(kTile), 0, s, L, nf, x, v, rho, alpha, kappa, xb, vb, kc,
                           dt, partials, go, nullptr);
    return hipGetLastError();
}

hipError_t launch_nonpressure_t(int model, const Lists& L, int64_t nf, float4* x, const float4* v, float4* vout,
                                const float* rho, Kern kc, float dt, float gx, float gy, float gz, float visc,
                                float* K, float* kappa, float warm_factor, bool setup_warm, hipStream_t s) {
    if (model == 1)
        TLAUNCH(k_nonpressure_t<1>, nf, x, v, vout, rho, kc, dt, gx, gy, gz, visc, K, kappa, warm_factor, setup_warm);
    if (model == 2)
        TLAUNCH(k_nonpressure_t<2>, nf, x, v, vout, rho, kc, dt, gx, gy, gz, visc, K, kappa, warm_factor, setup_warm);
    TLAUNCH(k_nonpressure_t<0>, nf, x, v, vout, rho, kc, dt, gx, gy, gz, visc, K, kappa, warm_factor, setup_warm);
}


hipError_t launch_rigid_force_t(const Lists& L, int64_t nf, const float4* x, const float* rho, const float* K,
                                const float* Kv, const float4* xb, const float4* vb, Kern kc, int32_t nbody,
                                const double* com, double* partials, HostStatus* host, hipStream_t s) {
    const uint32_t nblk = tile_blocks(L.ntiles);
    if (L.ntiles > 0)
        hipLaunchKernelGGL(k_rigid_force_t, dim3(nblk), dim3(kTile), 0, s, L, nf, x, rho, K, Kv, xb, vb, kc, nbody,
                           com, partials);
    hipLaunchKernelGGL(k_finish_rigid, dim3(1), dim3(kBlock), 0, s, partials, L.ntiles > 0 ? (int)nblk : 0, 6 * nbody,
                       host);
    return hipGetLastError();
}

hipError_t launch_visc_precond_t(const Lists& L, int64_t nf, const float4* x, const float* rho, Kern kc, float dt,
                                 float mu, float* Pinv, hipStream_t s) {
    TLAUNCH(k_visc_precond_t, nf, x, rho, kc, dt, mu, Pinv);
}

hipError_t launch_visc_matvec_t(const Lists& L, int64_t nf, const float4* x, const float* rho, const float4* p,
                                float4* Mp, Kern kc, float dt, float mu, hipStream_t s) {
    TLAUNCH(k_visc_matvec_t, nf, x, rho, p, Mp, kc, dt, mu);
}

}  // namespace sph
