// sph_kernels.hip -- gfx950 kernels of the DFSPH time step.
//
// One lane per particle, 256-lane workgroups, particles kept in (cell key,
// id) order so that neighbour gathers hit the XCD-local L2.  Workgroup ids are
// remapped so that each of the 8 XCDs walks one contiguous eighth of the
// particle range (hardware dispatch is round-robin over XCDs).
//
// The only integer decisions taken in floating point -- cell keys and the
// neighbour predicate -- use explicit non-contracted FP32 so that they are
// bit-exact with any IEEE implementation of the same formula.  Sums over
// neighbours are FP32; every reduction that decides convergence or
// accumulates a rigid-body force is FP64 in a fixed order (no float
// atomics), so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "sph_internal.h"
#include "sph_device.h"

namespace sph {
namespace {

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ counting sort
// Cell key and a provisional rank within the cell (the rank order is erased by
// the per-cell id sort).  The lanes of a wave that share a key (consecutive
// particles are mostly in the same cell, the input being last step's order)
// take one atomic per distinct key and rank among themselves by lane.
__global__ void k_keys_hist(const float4* __restrict__ x, int64_t n, Grid g, uint32_t* __restrict__ key,
                            uint32_t* __restrict__ slot, uint32_t* __restrict__ count) {
    const int64_t i = particle_index();
    const bool valid = i < n;
    uint32_t k = 0;
    if (valid) {
        k = cell_key(g, x[i]);
        key[i] = k;
    }
    // group the wave's lanes by key (the first lane of a group leads it),
    // then every leader adds its group's size with one atomic, all at once
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t pending = __ballot(valid);
    uint32_t rank = 0, group = 0;
    int leader_of = lane;
    while (pending) {   // wave-uniform
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const uint32_t kl = (uint32_t)__shfl((int)k, leader, 64);
        const uint64_t same = __ballot(valid && k == kl) & pending;
        if ((same >> lane) & 1ull) {
            rank = (uint32_t)__popcll(same & below);
            leader_of = leader;
        }
        if (lane == leader) group = (uint32_t)__popcll(same);
        pending &= ~same;
    }
    uint32_t base = 0;
    if (valid && leader_of == lane) base = atomicAdd(count + k, group);
    base = (uint32_t)__shfl((int)base, leader_of, 64);
    if (valid) slot[i] = base + rank;
}

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

// Exclusive scan of one 4096-entry tile; writes the tile total to partials.
__global__ void k_scan_local(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ out,
                             uint32_t* __restrict__ partials) {
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t wsum[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
        const int64_t gi = base + k;
        tile[k] = gi < n ? in[gi] : 0u;
    }
    __syncthreads();
    uint32_t local[kScanItems];
    uint32_t sum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        local[k] = sum;
        sum += tile[threadIdx.x * kScanItems + k];
    }
    const int lane = threadIdx.x & 63;
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wbase += wsum[w];
    const uint32_t excl = wbase + incl - sum;
    for (int k = 0; k < kScanItems; ++k) tile[threadIdx.x * kScanItems + k] = excl + local[k];
    __syncthreads();
    for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
        const int64_t gi = base + k;
        if (gi < n) out[gi] = tile[k];
    }
    if (threadIdx.x == kBlock - 1) partials[blockIdx.x] = excl + sum;
}

__global__ void k_scan_add(uint32_t* __restrict__ out, int64_t n, const uint32_t* __restrict__ tile_base,
                           const uint32_t* __restrict__ total) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] += tile_base[i / kScanTile];
    if (i == n) out[n] = *total;
}

__global__ void k_scatter(const uint32_t* __restrict__ key, const uint32_t* __restrict__ slot,
                          const uint32_t* __restrict__ start, int64_t n, uint32_t* __restrict__ src) {
    const int64_t i = particle_index();
    if (i >= n) return;
    src[start[key[i]] + slot[i]] = (uint32_t)i;
}

// Insertion sort of each cell's entries by particle id (cells hold ~8).
// Cells above 4096 entries are left unsorted and flagged (bit 1).
__global__ void k_cell_sort(const uint32_t* __restrict__ start, int64_t ncell, uint32_t* __restrict__ src,
                            const int32_t* __restrict__ id, uint32_t* flags) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    const uint32_t b = start[c], e = start[c + 1];
    if (e - b < 2) return;
    if (e - b > 4096) {
        atomicOr(flags, 2u);
        return;
    }
    for (uint32_t p = b + 1; p < e; ++p) {
        const uint32_t s = src[p];
        const int32_t key = id[s];
        uint32_t q = p;
        while (q > b && id[src[q - 1]] > key) {
            src[q] = src[q - 1];
            --q;
        }
        src[q] = s;
    }
}

// Reorder the per-particle state by the permutation; x.w = Kv / rho, the
// previous step's divergence stiffness over its density (the next warm start).
__global__ void k_gather_fluid(const uint32_t* __restrict__ src, int64_t n, const float4* __restrict__ x,
                               const float4* __restrict__ v, const float* __restrict__ K,
                               const float* __restrict__ Kv, const float* __restrict__ rho,
                               const int32_t* __restrict__ id, const float4* __restrict__ dv, float4* __restrict__ xo,
                               float4* __restrict__ vo, float* __restrict__ Ko, float* __restrict__ Kvo,
                               float* __restrict__ rhoo, int32_t* __restrict__ ido, float4* __restrict__ dvo) {
    const int64_t i = particle_index();
    if (i >= n) return;
    const uint32_t s = src[i];
    const float kv = Kv[s], r = rho[s];
    const float4 xs = x[s];
    xo[i] = make_float4(xs.x, xs.y, xs.z, kv / r);
    vo[i] = v[s];
    Ko[i] = K[s];
    Kvo[i] = kv;
    rhoo[i] = r;
    ido[i] = id[s];
    if (dv != nullptr) dvo[i] = dv[s];
}

__global__ void k_gather_boundary(const uint32_t* __restrict__ src, int64_t n, const float4* __restrict__ x,
                                  const float4* __restrict__ v, const int32_t* __restrict__ id,
                                  float4* __restrict__ xo, float4* __restrict__ vo, int32_t* __restrict__ ido) {
    const int64_t i = particle_index();
    if (i >= n) return;
    const uint32_t s = src[i];
    xo[i] = x[s];
    vo[i] = v[s];
    ido[i] = id[s];
}

// ------------------------------------------------------------------ neighbour lists
// Walk the 27-cell stencil (dz, dy outer; the contiguous cx-1..cx+1 run of
// sorted particles inner), which yields ascending sorted indices; fluid
// rows first, then boundary rows.
__global__ void __launch_bounds__(kBlock) k_nbr_build(
    const float4* __restrict__ x, int64_t nf, const float4* __restrict__ xb, const uint32_t* __restrict__ start_f,
    const uint32_t* __restrict__ start_b, Grid g, uint32_t* __restrict__ nlist, uint32_t* __restrict__ ncnt,
    int32_t capf, uint32_t* __restrict__ blist, uint32_t* __restrict__ bcnt, int32_t capb, uint32_t* flags,
    unsigned long long* __restrict__ stats) {
    __shared__ float4 win_all[kBlock / 64][kWinSlots];
    float4* win = win_all[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int64_t i = particle_index();
    const bool valid = i < nf;
    uint32_t total = 0xffffffffu, fl = 0;
    // the wave's particles usually lie in consecutive cells of one row of the
    // grid (sorted order, x fastest): then each of the nine stencil rows is
    // one contiguous window of sorted particles for the whole wave, staged in
    // LDS with coalesced loads, and the lanes test their candidates there
    const float4 xi = valid ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int32_t cx = cell_coord(xi.x, g.o[0], g.inv, g.n[0]);
    const int32_t cy = cell_coord(xi.y, g.o[1], g.inv, g.n[1]);
    const int32_t cz = cell_coord(xi.z, g.o[2], g.inv, g.n[2]);
    const int32_t x0 = cx > 0 ? cx - 1 : 0, x1 = cx < g.n[0] - 1 ? cx + 1 : g.n[0] - 1;
    const unsigned long long vmask = __ballot(valid);
    const int src = vmask ? __ffsll((long long)vmask) - 1 : 0;
    const int32_t cy0 = __shfl(cy, src, 64), cz0 = __shfl(cz, src, 64);
    const bool one_row = vmask != 0ull && __all(!valid || (cy == cy0 && cz == cz0));
    int32_t xlo = valid ? x0 : 0x7fffffff, xhi = valid ? x1 : -1;
    for (int off = 32; off > 0; off >>= 1) {
        xlo = min(xlo, __shfl_xor(xlo, off, 64));
        xhi = max(xhi, __shfl_xor(xhi, off, 64));
    }
    uint32_t nfc = 0, nbc = 0;
    uint4 fbuf = make_uint4(0u, 0u, 0u, 0u), bbuf = make_uint4(0u, 0u, 0u, 0u);
    uint4* fchunk = reinterpret_cast<uint4*>(nlist) + i;   // chunk 0 of particle i
    uint4* bchunk = reinterpret_cast<uint4*>(blist) + i;
    // the nine rows' candidate ranges, all loads issued before the scans
    // (a row outside the grid reads row 0 and is made empty)
    uint32_t fb[9], fe[9], bb[9], be[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const int32_t z = cz + r / 3 - 1, y = cy + r % 3 - 1;
        const bool ok = valid && z >= 0 && z < g.n[2] && y >= 0 && y < g.n[1];
        const int64_t row = ok ? (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z) : 0;
        fb[r] = start_f[row + x0];
        fe[r] = start_f[row + x1 + 1];
        bb[r] = start_b[row + x0];
        be[r] = start_b[row + x1 + 1];
        if (!ok) fe[r] = fb[r], be[r] = bb[r];
    }
    // only the middle row (dy = dz = 0) holds the particle itself
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        bool staged = false;
        if (one_row) {   // wave-uniform
            const int32_t z = cz0 + r / 3 - 1, y = cy0 + r % 3 - 1;
            const bool ok = z >= 0 && z < g.n[2] && y >= 0 && y < g.n[1];
            const int64_t row = ok ? (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z) : 0;
            const uint32_t wb = ok ? start_f[row + xlo] : 0u, we = ok ? start_f[row + xhi + 1] : 0u;
            if (we - wb <= kWinCand) {   // the window holds every lane's range [fb, fe)
                wave_lds_sync();   // the previous row's reads are done
                for (uint32_t t = lane; t < we - wb; t += 64) win[win_slot(t)] = x[wb + t];
                wave_lds_sync();
                if (r == 4)
                    scan_window<true>(win, wb, fb[r], fe[r], xi, (uint32_t)i, g.h2, fchunk, nf, capf, nfc, fbuf);
                else
                    scan_window<false>(win, wb, fb[r], fe[r], xi, 0u, g.h2, fchunk, nf, capf, nfc, fbuf);
                staged = true;
            }
        }
        if (!staged) {
            if (r == 4)
                scan_candidates<true>(x, fb[r], fe[r], xi, (uint32_t)i, g.h2, fchunk, nf, capf, nfc, fbuf);
            else
                scan_candidates<false>(x, fb[r], fe[r], xi, 0u, g.h2, fchunk, nf, capf, nfc, fbuf);
        }
    }
#pragma unroll
    for (int r = 0; r < 9; ++r)
        scan_candidates<false>(xb, bb[r], be[r], xi, 0u, g.h2, bchunk, nf, capb, nbc, bbuf);
    if (valid) {
        list_flush(fchunk, capf, nfc, fbuf);
        list_flush(bchunk, capb, nbc, bbuf);
        // stored counts never exceed the capacity, so readers stay in bounds
        ncnt[i] = min(nfc, (uint32_t)capf);
        bcnt[i] = min(nbc, (uint32_t)capb);
        if (nfc > (uint32_t)capf || nbc > (uint32_t)capb) atomicOr(flags, 1u);
        total = nfc + nbc;
        fl = nfc;
    }
    // neighbour-count statistics: min, max, sum (integer atomics, exact)
    uint32_t mn = total, mx = (i < nf) ? total : 0u;
    unsigned long long sm = (i < nf) ? total : 0ull, sf = fl;
    for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, (uint32_t)__shfl_down((int)mn, off, 64));
        mx = max(mx, (uint32_t)__shfl_down((int)mx, off, 64));
        sm += __shfl_down(sm, off, 64);
        sf += __shfl_down(sf, off, 64);
    }
    __shared__ unsigned long long ws[kBlock / 64][4];
    if ((threadIdx.x & 63) == 0) {
        ws[threadIdx.x >> 6][0] = mn;
        ws[threadIdx.x >> 6][1] = mx;
        ws[threadIdx.x >> 6][2] = sm;
        ws[threadIdx.x >> 6][3] = sf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = ws[0][0], b = ws[0][1], c = ws[0][2], d = ws[0][3];
        for (int w = 1; w < kBlock / 64; ++w) {
            a = min(a, ws[w][0]);
            b = max(b, ws[w][1]);
            c += ws[w][2];
            d += ws[w][3];
        }
        unsigned long long* o = stats + (size_t)kNStats * blockIdx.x;
        o[0] = a;
        o[1] = b;
        o[2] = c;
        o[3] = d;
    }
}

// Akinci boundary mass, Eq. (11): Psi_b = rho0 / (W(0) + sum_{k != b} W_bk) over
// all boundary particles within h; stored in xb[b].w.
__global__ void k_boundary_psi(float4* __restrict__ xb, int64_t nb, const uint32_t* __restrict__ start_b, Grid g,
                               Kern kc) {
    const int64_t i = particle_index();
    if (i >= nb) return;
    const float4 xi = xb[i];
    const int32_t cx = cell_coord(xi.x, g.o[0], g.inv, g.n[0]);
    const int32_t cy = cell_coord(xi.y, g.o[1], g.inv, g.n[1]);
    const int32_t cz = cell_coord(xi.z, g.o[2], g.inv, g.n[2]);
    const int32_t x0 = cx > 0 ? cx - 1 : 0, x1 = cx < g.n[0] - 1 ? cx + 1 : g.n[0] - 1;
    float s = kc.k;
    for (int32_t dz = -1; dz <= 1; ++dz) {
        const int32_t z = cz + dz;
        if (z < 0 || z >= g.n[2]) continue;
        for (int32_t dy = -1; dy <= 1; ++dy) {
            const int32_t y = cy + dy;
            if (y < 0 || y >= g.n[1]) continue;
            const int64_t row = (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z);
            const uint32_t b = start_b[row + x0], e = start_b[row + x1 + 1];
            for (uint32_t k = b; k < e; ++k) {
                if ((int64_t)k == i) continue;
                const float4 xk = xb[k];
                const float d2 = dist2_exact(xi, xk);
                if (d2 < g.h2) s += kernel_W(d2, kc);
            }
        }
    }
    xb[i].w = kc.rho0 / s;
}

// ------------------------------------------------------------------ the step
// |v|^2 as fl32((vx^2 + vy^2) + vz^2), every product and sum rounded
__device__ __forceinline__ float speed2(float4 a) {
#pragma clang fp contract(off)
    const float xx = a.x * a.x, yy = a.y * a.y, zz = a.z * a.z;
    const float s = xx + yy;
    return s + zz;
}

// the workgroup's maximum of m >= 0 into out_bits[blockIdx.x]
__device__ __forceinline__ void block_max_bits(float m, uint32_t* out_bits) {
    uint32_t bits = __float_as_uint(m);   // non-negative floats order as integers
    for (int off = 32; off > 0; off >>= 1) bits = max(bits, (uint32_t)__shfl_down((int)bits, off, 64));
    __shared__ uint32_t ws[kBlock / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = ws[0];
        for (int w = 1; w < kBlock / 64; ++w) m = max(m, ws[w]);
        out_bits[blockIdx.x] = m;
    }
}

__global__ void k_max_v2(const float4* __restrict__ v, int64_t n, uint32_t* out_bits) {
    const int64_t i = particle_index();
    block_max_bits(i < n ? speed2(v[i]) : 0.0f, out_bits);
}

// The neighbour sums below run L lanes per particle (group_particle,
// for_each_nbr_l, group_sum); the launchers pick L per pass.

// Density with the Akinci boundary term, Eq. (12), and the DFSPH factor
// alpha = rho / (|sum_F m gradW + sum_B Psi gradW|^2 + sum_F |m gradW|^2).
// Also saves the step's input velocity and stores the particle volume m/rho
// in v.w (the XSPH pass then gathers a neighbour's velocity and volume in
// one load, with no division per neighbour).  WARM:
// the divergence solve's warm start in the same neighbour walk: its
// stiffness over density, warm_factor Kv_prev / rho_prev (x.w, from the sort),
// does not depend on this step's density, so its pressure (Eq. 7 with the
// Eq. 13 boundary term) is applied here, and Kv starts at that times rho.
// DIN: the walk also sums the density change rate of the step's input
// velocity (Eq. 9 in the DFSPH form, with the boundary velocities vb when
// given) into din, a feature of the learned warm start; neighbours then read
// v during the pass, so the updated velocities go to vout (a different
// buffer), else vout == v.
template <int L, bool WARM, bool DIN>
__global__ void __launch_bounds__(kBlock) k_density_alpha(
    int64_t nf, float4* __restrict__ x, const float4* v, float4* vout, const uint32_t* __restrict__ nlist,
    const uint32_t* __restrict__ ncnt, const float4* __restrict__ xb, const float4* __restrict__ vb,
    const uint32_t* __restrict__ blist, const uint32_t* __restrict__ bcnt, Kern kc, float* __restrict__ rho,
    float* __restrict__ alpha, float4* __restrict__ v_in, float* __restrict__ Kv, float dt, float warm_factor,
    float pci_c, float* __restrict__ din) {
    int q;
    const int64_t i = group_particle<L>(q);
    if (i >= nf) return;   // whole groups leave together
    const float4 xi = x[i];
    const float4 vi0 = DIN ? v[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float kri = WARM ? warm_factor * xi.w : 0.0f;   // x.w = Kv_prev / rho_prev (from the sort)
    float r = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, sq = 0.f;
    float px = 0.f, py = 0.f, pz = 0.f, dv = 0.f;
    for_each_nbr_l<L>(nlist, nf, i, q, ncnt[i], [&](uint32_t j) {
        const float4 xj = x[j];
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        r += kc.m * kernel_W(r2, kc);
        const float g = grad_factor(r2, kc);
        const float F = kc.m * g;
        const float ax = F * dx, ay = F * dy, az = F * dz;
        gx += ax; gy += ay; gz += az;
        sq += ax * ax + ay * ay + az * az;
        if (WARM) {
            const float c = (kri + warm_factor * xj.w) * g;
            px += c * dx; py += c * dy; pz += c * dz;
        }
        if (DIN) {
            const float4 vj = v[j];
            dv += g * ((vi0.x - vj.x) * dx + (vi0.y - vj.y) * dy + (vi0.z - vj.z) * dz);
        }
    });
    float rb = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
    float pbx = 0.f, pby = 0.f, pbz = 0.f, dvb = 0.f;
    for_each_nbr_l<L>(blist, nf, i, q, bcnt[i], [&](uint32_t kk) {
        const float4 xk = xb[kk];
        const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        rb += xk.w * kernel_W(r2, kc);
        const float g = grad_factor(r2, kc);
        const float F = xk.w * g;
        bx += F * dx; by += F * dy; bz += F * dz;
        if (WARM) {
            const float c = xk.w * kri * g;
            pbx += c * dx; pby += c * dy; pbz += c * dz;
        }
        if (DIN) {
            const float4 vk = vb ? vb[kk] : make_float4(0.f, 0.f, 0.f, 0.f);
            dvb += F * ((vi0.x - vk.x) * dx + (vi0.y - vk.y) * dy + (vi0.z - vk.z) * dz);
        }
    });
    // self term, fluid sum, boundary sum
    const float rr = (kc.m * kc.k + group_sum<L>(r)) + group_sum<L>(rb);
    gx = group_sum<L>(gx) + group_sum<L>(bx);
    gy = group_sum<L>(gy) + group_sum<L>(by);
    gz = group_sum<L>(gz) + group_sum<L>(bz);
    sq = group_sum<L>(sq);
    if (WARM) {
        px = group_sum<L>(px) * kc.m + group_sum<L>(pbx);
        py = group_sum<L>(py) * kc.m + group_sum<L>(pby);
        pz = group_sum<L>(pz) * kc.m + group_sum<L>(pbz);
    }
    if (DIN) dv = group_sum<L>(dv) * kc.m + group_sum<L>(dvb);
    if (q != 0) return;
    if (DIN) din[i] = dv;
    const float D = gx * gx + gy * gy + gz * gz + sq;
    rho[i] = rr;
    // PCISPH (pci_c > 0): the prototype factor c / rho replaces alpha
    float a = D > kc.d_min ? rr / D : 0.0f;
    if (kc.alpha_max > 0.0f) a = fminf(a, kc.alpha_max);
    alpha[i] = pci_c > 0.0f ? pci_c / rr : a;
    float4 vi = v[i];
    v_in[i] = vi;
    if (WARM) {
        vi.x -= dt * px; vi.y -= dt * py; vi.z -= dt * pz;
    }
    vout[i] = make_float4(vi.x, vi.y, vi.z, kc.m / rr);
    Kv[i] = WARM ? kri * rr : 0.0f;
}

// Pressure velocity update (Eq. 7 with p/rho^2 = kappa/rho, the boundary term
// of Eq. 13 using the particle's own pressure): kappa/rho comes from x.w.
template <int L>
__global__ void __launch_bounds__(kBlock) k_pressure_update(
    int64_t nf, const float4* __restrict__ x, float4* __restrict__ v, const float* __restrict__ kappa,
    float* __restrict__ Kacc, float* __restrict__ kappa_last, const uint32_t* __restrict__ nlist,
    const uint32_t* __restrict__ ncnt, const float4* __restrict__ xb, const uint32_t* __restrict__ blist,
    const uint32_t* __restrict__ bcnt, Kern kc, float dt, const int32_t* __restrict__ go) {
    if (go != nullptr && *go == 0) return;
    int q;
    const int64_t i = group_particle<L>(q);
    if (i >= nf) return;
    const float4 xi = x[i];
    const float kri = xi.w;
    float ax = 0.f, ay = 0.f, az = 0.f;
    for_each_nbr_l<L>(nlist, nf, i, q, ncnt[i], [&](uint32_t j) {
        const float4 xj = x[j];
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float c = (kri + xj.w) * grad_factor(r2, kc);
        ax += c * dx; ay += c * dy; az += c * dz;
    });
    float bx = 0.f, by = 0.f, bz = 0.f;
    for_each_nbr_l<L>(blist, nf, i, q, bcnt[i], [&](uint32_t kk) {
        const float4 xk = xb[kk];
        const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float c = xk.w * kri * grad_factor(r2, kc);
        bx += c * dx; by += c * dy; bz += c * dz;
    });
    ax = group_sum<L>(ax) * kc.m + group_sum<L>(bx);
    ay = group_sum<L>(ay) * kc.m + group_sum<L>(by);
    az = group_sum<L>(az) * kc.m + group_sum<L>(bz);
    if (q != 0) return;
    float4 vi = v[i];
    vi.x -= dt * ax; vi.y -= dt * ay; vi.z -= dt * az;
    v[i] = vi;
    const float ki = kappa[i];
    Kacc[i] += ki;
    if (kappa_last) kappa_last[i] = ki;
}

// Divergence d_i = sum_F m (v_i - v_j).gradW + sum_B Psi (v_i - v_k).gradW
// (Eq. 6 in the DFSPH form, Eq. 9 for the predicted density), the next
// stiffness, and the FP64 sum of the clamped error.
template <int MODE, int L>
__global__ void __launch_bounds__(kBlock) k_predict(
    int64_t nf, float4* __restrict__ x, const float4* __restrict__ v, const float* __restrict__ rho,
    const float* __restrict__ alpha, float* __restrict__ kappa, const uint32_t* __restrict__ nlist,
    const uint32_t* __restrict__ ncnt, const float4* __restrict__ xb, const float4* __restrict__ vb,
    const uint32_t* __restrict__ blist, const uint32_t* __restrict__ bcnt, Kern kc, float dt,
    double* __restrict__ partials, const int32_t* __restrict__ go, float* __restrict__ dout) {
    if (go != nullptr && *go == 0) return;
    int q;
    const int64_t i = group_particle<L>(q);
    double e = 0.0;
    float em = 0.0f;   // the density solve's largest clamped deviation (MODE 1)
    if (i < nf) {   // whole groups
        const float4 xi = x[i];
        const float4 vi = v[i];
        float d = 0.f;
        for_each_nbr_l<L>(nlist, nf, i, q, ncnt[i], [&](uint32_t j) {
            const float4 xj = x[j];
            const float4 vj = v[j];
            const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            d += grad_factor(r2, kc) * ((vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz);
        });
        float db = 0.f;
        for_each_nbr_l<L>(blist, nf, i, q, bcnt[i], [&](uint32_t kk) {
            const float4 xk = xb[kk];
            const float4 vk = vb ? vb[kk] : make_float4(0.f, 0.f, 0.f, 0.f);   // null: all boundaries at rest
            const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            db += xk.w * grad_factor(r2, kc) * ((vi.x - vk.x) * dx + (vi.y - vk.y) * dy + (vi.z - vk.z) * dz);
        });
        d = group_sum<L>(d) * kc.m + group_sum<L>(db);
        if (q == 0) {
            const float ri = rho[i];
            float kap;
            if (MODE == 0) {
                if (dout) dout[i] = d;
                const float ep = fmaxf(d, 0.0f);
                kap = ep * alpha[i] / dt;
                e = err_term(d, ep);
            } else {
                const float dev = (ri - kc.rho0) + dt * d;
                const float ep = fmaxf(dev, 0.0f);
                kap = ep * alpha[i] / (dt * dt);
                e = err_term(dev, ep);
                em = ep;
            }
            kappa[i] = kap;
            x[i].w = kap / ri;
        }
    }
    const double bs = block_sum(e);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    if (MODE == 1) {   // the workgroup maxima follow the sums (read when the solve bounds the maximum)
        const float bm = block_max(em);
        if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = (double)bm;
    }
}

// Non-pressure accelerations (Algorithm 1, first lines): v* = v + dt g plus
// XSPH (model 1) or the explicit Laplacian of Eq. (15) (model 2); and the
// set-up of the density warm start (kappa = warm_factor K, K = 0, x.w = kappa/rho).
// PRESS: the same pass also applies the pressure of the stiffness kappa/rho
// already in x.w (the density solve's warm start, or WCSPH's equation of
// state), as k_pressure_update would right after it: v* -= dt (Eq. 7 with the
// Eq. 13 boundary term), K += kappa, kappa_last = kappa.  Both sums read the
// step's v and x, so one neighbour walk serves them.
// DIV: the walk also takes the divergence-free solve's first error pass
// (k_predict, mode 0) on the same v: D rho/Dt (Eq. 4 with the boundary
// term), its stiffness kappa_v = max(D rho/Dt, 0) alpha / dt and the FP64
// per-workgroup partials of the error.  kappa_v and kappa_v/rho go to
// dc.kvs when PRESS (x.w is being read as the warm start's kappa/rho), else
// to kappa and x.w as k_predict writes them; D rho/Dt to dc.dout if given.
template <int MODEL, int L, bool PRESS, bool DIV>
__global__ void __launch_bounds__(kBlock) k_nonpressure(
    int64_t nf, float4* __restrict__ x, const float4* __restrict__ v, float4* __restrict__ vout,
    const float* __restrict__ rho, const uint32_t* __restrict__ nlist, const uint32_t* __restrict__ ncnt,
    Kern kc, float dt, float gx, float gy, float gz, float visc, float* __restrict__ K, float* __restrict__ kappa,
    float warm_factor, bool setup_warm, const float4* __restrict__ xb, const uint32_t* __restrict__ blist,
    const uint32_t* __restrict__ bcnt, float* __restrict__ kappa_last, DivCheck dc) {
    int q;
    const int64_t i = group_particle<L>(q);
    double e = 0.0;
    if (i < nf) {   // whole groups
        const float4 xi = x[i];
        const float4 vi = v[i];
        const float kri = xi.w;   // kappa/rho (PRESS)
        float ax = 0.f, ay = 0.f, az = 0.f;
        float px = 0.f, py = 0.f, pz = 0.f;
        float dd = 0.f, db = 0.f;
        if (MODEL == 1 || MODEL == 2 || PRESS || DIV) {
            const float eps2 = 0.01f * kc.h * kc.h;
            for_each_nbr_l<L>(nlist, nf, i, q, ncnt[i], [&](uint32_t j) {
                const float4 xj = x[j];
                const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                float4 vj;
                if (MODEL == 1 || MODEL == 2 || DIV) vj = v[j];
                if (MODEL == 1 || MODEL == 2) {
                    const float mj = vj.w;   // v.w = m / rho (density pass)
                    if (MODEL == 1) {
                        const float c = mj * kernel_W(r2, kc);
                        ax += c * (vj.x - vi.x); ay += c * (vj.y - vi.y); az += c * (vj.z - vi.z);
                    } else {
                        const float vx = (vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz;
                        const float c = mj * vx / (r2 + eps2) * grad_factor(r2, kc);
                        ax += c * dx; ay += c * dy; az += c * dz;
                    }
                }
                if (PRESS) {
                    const float c = (kri + xj.w) * grad_factor(r2, kc);
                    px += c * dx; py += c * dy; pz += c * dz;
                }
                if (DIV)
                    dd += grad_factor(r2, kc) * ((vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz);
            });
            if (MODEL == 1 || MODEL == 2) {
                ax = group_sum<L>(ax); ay = group_sum<L>(ay); az = group_sum<L>(az);
            }
        }
        if (PRESS || DIV) {
            float bx = 0.f, by = 0.f, bz = 0.f;
            for_each_nbr_l<L>(blist, nf, i, q, bcnt[i], [&](uint32_t kk) {
                const float4 xk = xb[kk];
                const float dx = xi.x - xk.x, dy = xi.y - xk.y, dz = xi.z - xk.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                if (PRESS) {
                    const float c = xk.w * kri * grad_factor(r2, kc);
                    bx += c * dx; by += c * dy; bz += c * dz;
                }
                if (DIV) {
                    const float4 vk = dc.vb ? dc.vb[kk] : make_float4(0.f, 0.f, 0.f, 0.f);
                    db += xk.w * grad_factor(r2, kc) * ((vi.x - vk.x) * dx + (vi.y - vk.y) * dy + (vi.z - vk.z) * dz);
                }
            });
            if (PRESS) {
                px = group_sum<L>(px) * kc.m + group_sum<L>(bx);
                py = group_sum<L>(py) * kc.m + group_sum<L>(by);
                pz = group_sum<L>(pz) * kc.m + group_sum<L>(bz);
            }
            if (DIV) dd = group_sum<L>(dd) * kc.m + group_sum<L>(db);
        }
        if (q == 0) {
            float s = 0.f;
            if (MODEL == 1) s = visc;
            if (MODEL == 2) s = dt * visc * 2.0f * (3 + 2);
            float4 o;
            o.x = vi.x + dt * gx + s * ax;
            o.y = vi.y + dt * gy + s * ay;
            o.z = vi.z + dt * gz + s * az;
            o.w = 0.f;
            if (PRESS) {
                o.x -= dt * px; o.y -= dt * py; o.z -= dt * pz;
                const float ki = kappa[i];
                K[i] += ki;
                if (kappa_last) kappa_last[i] = ki;
            }
            vout[i] = o;
            if (!PRESS && setup_warm) {
                const float k0 = warm_factor * K[i];
                kappa[i] = k0;
                K[i] = 0.0f;
                x[i].w = k0 / rho[i];
            }
            if (DIV) {
                const float ri = rho[i];
                if (dc.dout) dc.dout[i] = dd;
                const float ep = fmaxf(dd, 0.0f);
                const float kap = ep * dc.alpha[i] / dt;
                e = err_term(dd, ep);
                if (PRESS) {
                    dc.kvs[i] = make_float2(kap, kap / ri);
                } else {
                    kappa[i] = kap;
                    x[i].w = kap / ri;
                }
            }
        }
    }
    if (DIV) {
        const double bs = block_sum(e);
        if (threadIdx.x == 0) dc.partials[blockIdx.x] = bs;
    }
}

// After a folded divergence check (k_nonpressure with PRESS and DIV) whose
// error calls for iterations: the state the separate check would have left
// for them (kappa = kappa_v, x.w = kappa_v/rho) and the K the warm start's
// set-up had saved.
__global__ void k_div_resume(int64_t nf, float4* __restrict__ x, float* __restrict__ kappa, float* __restrict__ K,
                             const float2* __restrict__ kvs, const float* __restrict__ Ksaved) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float2 kv = kvs[i];
    kappa[i] = kv.x;
    x[i].w = kv.y;
    K[i] = Ksaved[i];
}

// Learned warm start, features of each particle at the start of the density
// solve, from per-particle fields: (rho - rho0)/rho0, dt d/rho0 with d the
// density change rate of the step's input velocity (from the density pass),
// (n_f + n_b)/26, K_prev dt^2/(alpha rho0), alpha/alpha_ref.
__global__ void k_features(int64_t nf, const float* __restrict__ rho, const float* __restrict__ alpha,
                           const float* __restrict__ K, const uint32_t* __restrict__ ncnt,
                           const uint32_t* __restrict__ bcnt, const float* __restrict__ d, Kern kc, float dt,
                           float alpha_ref, float* __restrict__ feat) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float a = alpha[i];
    float* f = feat + 5 * i;
    f[0] = (rho[i] - kc.rho0) / kc.rho0;
    f[1] = dt * d[i] / kc.rho0;
    f[2] = (float)(ncnt[i] + bcnt[i]) / 26.0f;
    f[3] = a > 0.0f ? K[i] * dt * dt / (a * kc.rho0) : 0.0f;
    f[4] = a / alpha_ref;
}

// WCSPH equation of state (Sec. 3.4.1): p = k ((rho/rho0)^gamma - 1), clamped
// at zero; kappa = p/rho (so p/rho^2 = kappa/rho as in the DFSPH passes),
// x.w = kappa/rho, K = 0 (the pressure pass accumulates kappa into it), and
// per-workgroup FP64 partials of max(rho - rho0, 0) for the reported error.
__global__ void k_eos(int64_t nf, float4* __restrict__ x, const float* __restrict__ rho, float* __restrict__ kappa,
                      float* __restrict__ K, Kern kc, float k, float gamma, double* __restrict__ partials) {
    const int64_t i = particle_index();
    double e = 0.0;
    if (i < nf) {
        const float r = rho[i];
        const float pw = powf(r / kc.rho0, gamma);
        const float p = fmaxf(k * (pw - 1.0f), 0.0f);
        const float kap = p / r;
        kappa[i] = kap;
        K[i] = 0.0f;
        x[i].w = kap / r;
        e = err_term(r - kc.rho0, fmaxf(r - kc.rho0, 0.0f));
    }
    const double bs = block_sum(e);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// K0 = max(0, y alpha rho0 / dt^2) from the MLP output y.
__global__ void k_warm_learned(int64_t nf, float4* __restrict__ x, const float* __restrict__ rho,
                               const float* __restrict__ alpha, const float* __restrict__ y, float* __restrict__ K,
                               float* __restrict__ kappa, float dt, float rho0) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float k0 = fmaxf(y[i] * alpha[i] * rho0 / (dt * dt), 0.0f);
    kappa[i] = k0;
    K[i] = 0.0f;
    x[i].w = k0 / rho[i];
}

// training target: the step's final density stiffness, K dt^2 / (alpha rho0)
__global__ void k_trace_target(int64_t nf, const float* __restrict__ alpha, const float* __restrict__ K, float dt,
                               float rho0, float* __restrict__ target) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float a = alpha[i];
    target[i] = a > 0.0f ? K[i] * dt * dt / (a * rho0) : 0.0f;
}

// x += dt v; out_bits (nullable): per-workgroup max |v|^2 of the new v, the
// next step's CFL input (as k_max_v2).  gate (nullable): nothing happens
// while *gate != 0 (queued behind a solve that may still be iterating).
__global__ void k_integrate(int64_t nf, float4* __restrict__ x, const float4* __restrict__ v, float dt,
                            uint32_t* out_bits, const int32_t* __restrict__ gate) {
    if (gate != nullptr && *gate != 0) return;
    const int64_t i = particle_index();
    float m = 0.0f;
    if (i < nf) {
        float4 xi = x[i];
        const float4 vi = v[i];
        xi.x += dt * vi.x; xi.y += dt * vi.y; xi.z += dt * vi.z;
        x[i] = xi;
        m = speed2(vi);
    }
    if (out_bits) block_max_bits(m, out_bits);
}

// Reaction on the rigid bodies (Eq. 14) from the step's total stiffness
// K + Kv: F_ik = m Psi_k ((K_i + Kv_i) / rho_i) gradW_ik, torque (x_k - c_b) x F.
// Pair terms in FP32, accumulation in FP64, fixed order.
// xw_scale > 0: the stiffness of one pressure pass, kappa/rho = xw_scale x.w
// (strong coupling), instead of the step's total (K + Kv)/rho; go (nullable):
// nothing happens when it reads 0.
__global__ void __launch_bounds__(kBlock) k_rigid_force(
    int64_t nf, const float4* __restrict__ x, const float* __restrict__ rho, const float* __restrict__ K,
    const float* __restrict__ Kv, const uint32_t* __restrict__ blist, const uint32_t* __restrict__ bcnt,
    const float4* __restrict__ xb, const float4* __restrict__ vb, Kern kc, int32_t nbody,
    const double* __restrict__ com, double* __restrict__ partials, float xw_scale, const int32_t* __restrict__ go) {
    if (go != nullptr && *go == 0) return;
    const int64_t i = particle_index();
    uint32_t nbk = 0;
    float4 xi = make_float4(0.f, 0.f, 0.f, 0.f);
    float base = 0.f;
    uint32_t mine = 0;   // bit b: a boundary neighbour of this particle belongs to body b
    if (i < nf) {
        nbk = bcnt[i];
        if (nbk) {
            xi = x[i];
            base = xw_scale > 0.0f ? kc.m * (xw_scale * xi.w) : kc.m * (K[i] + Kv[i]) / rho[i];
        }
        for (uint32_t k = 0; k < nbk; ++k) {
            const int32_t b = (int32_t)vb[blist[list_index(nf, i, k)]].w;
            if (b >= 0) mine |= 1u << b;
        }
    }
    // the bodies the workgroup touches (integer OR: exact); most workgroups
    // touch none and only store zeros
    for (int off = 32; off > 0; off >>= 1) mine |= (uint32_t)__shfl_xor((int)mine, off, 64);
    __shared__ uint32_t wmask[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wmask[threadIdx.x >> 6] = mine;
    __syncthreads();
    uint32_t touched = 0;
    for (int w = 0; w < kBlock / 64; ++w) touched |= wmask[w];
    const size_t nblk = gridDim.x;
    for (int32_t b = 0; b < nbody; ++b) {
        if (!((touched >> b) & 1u)) {
            if (threadIdx.x < 6) partials[(size_t)(6 * b + threadIdx.x) * nblk + blockIdx.x] = 0.0;
            continue;
        }
        double f[3] = {0.0, 0.0, 0.0}, t[3] = {0.0, 0.0, 0.0};
        if ((mine >> b) & 1u) {
            for (uint32_t k = 0; k < nbk; ++k) {
                const uint32_t kk = blist[list_index(nf, i, k)];
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
                t[0] += ry * Fz - rz * Fy;
                t[1] += rz * Fx - rx * Fz;
                t[2] += rx * Fy - ry * Fx;
            }
        }
        for (int c = 0; c < 3; ++c) {
            const double s0 = block_sum(f[c]);
            const double s1 = block_sum(t[c]);
            if (threadIdx.x == 0) {
                partials[(size_t)(6 * b + c) * nblk + blockIdx.x] = s0;
                partials[(size_t)(6 * b + 3 + c) * nblk + blockIdx.x] = s1;
            }
        }
    }
}

// Rigid boundary particles from the body pose: x_k = fl32(c + R r_k) and
// v_k = fl32(V + w x (x_k - c)), FP64 with no contraction.
__global__ void k_rigid_boundary(int64_t nb, float4* __restrict__ xb, float4* __restrict__ vb,
                                 const int32_t* __restrict__ bid, const double* __restrict__ local,
                                 const BodyPose* __restrict__ poses, const int32_t* __restrict__ go) {
#pragma clang fp contract(off)
    if (go != nullptr && *go == 0) return;
    const int64_t i = particle_index();
    if (i >= nb) return;
    float4 vk = vb[i];
    const int32_t b = (int32_t)vk.w;
    if (b < 0) return;
    const BodyPose& P = poses[b];
    const int64_t id = bid[i];
    const double l0 = local[3 * id], l1 = local[3 * id + 1], l2 = local[3 * id + 2];
    float xf[3];
    for (int a = 0; a < 3; ++a) {
        double t = P.R[3 * a] * l0 + P.R[3 * a + 1] * l1;
        t = t + P.R[3 * a + 2] * l2;
        xf[a] = (float)(P.com[a] + t);
    }
    const double rx = (double)xf[0] - P.com[0], ry = (double)xf[1] - P.com[1], rz = (double)xf[2] - P.com[2];
    const double wx = P.omega[1] * rz - P.omega[2] * ry;
    const double wy = P.omega[2] * rx - P.omega[0] * rz;
    const double wz = P.omega[0] * ry - P.omega[1] * rx;
    float4 xk = xb[i];
    xk.x = xf[0]; xk.y = xf[1]; xk.z = xf[2];
    xb[i] = xk;
    vk.x = (float)(P.vel[0] + wx);
    vk.y = (float)(P.vel[1] + wy);
    vk.z = (float)(P.vel[2] + wz);
    vb[i] = vk;
}

// ------------------------------------------------------------------ implicit viscosity
// (A v)_i = sum_j 10 mu m / (rho_i rho_j) (x_ij.(v_i - v_j)) / (|x_ij|^2 + 0.01 h^2) gradW_ij
// Every CG vector carries the particle volume m/rho in its w component
// (k_cg_start copies it from v.w), so a neighbour costs two gathers, x_j and
// p_j.  With `partials` the
// pass also stores the per-workgroup FP64 sums of p.(M p) for the CG step.
template <int L>
__global__ void __launch_bounds__(kBlock) k_visc_matvec(
    int64_t nf, const float4* __restrict__ x, const float4* __restrict__ p, float4* __restrict__ Mp,
    const uint32_t* __restrict__ nlist, const uint32_t* __restrict__ ncnt, Kern kc, float dt, float mu,
    const int32_t* __restrict__ go, double* __restrict__ partials) {
    if (go != nullptr && *go == 0) return;
    int q;
    const int64_t i = group_particle<L>(q);
    double e = 0.0;
    if (i < nf) {   // whole groups
        const float4 xi = x[i];
        const float4 pi = p[i];
        const float eps2 = 0.01f * kc.h * kc.h;
        float ax = 0.f, ay = 0.f, az = 0.f;
        for_each_nbr_l<L>(nlist, nf, i, q, ncnt[i], [&](uint32_t j) {
            const float4 xj = x[j];
            const float4 pj = p[j];
            const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float xv = (pi.x - pj.x) * dx + (pi.y - pj.y) * dy + (pi.z - pj.z) * dz;
            const float c = xv * pj.w / (kc.m * (r2 + eps2)) * grad_factor(r2, kc);
            ax += c * dx; ay += c * dy; az += c * dz;
        });
        ax = group_sum<L>(ax);
        ay = group_sum<L>(ay);
        az = group_sum<L>(az);
        if (q == 0) {
            const float s = dt * 10.0f * mu * pi.w;
            const float4 o = make_float4(pi.x - s * ax, pi.y - s * ay, pi.z - s * az, pi.w);
            Mp[i] = o;
            e = (double)pi.x * o.x + (double)pi.y * o.y + (double)pi.z * o.z;
        }
    }
    if (partials != nullptr) {
        const double bs = block_sum(e);
        if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    }
}

// Inverse of the 3x3 diagonal block I - dt A_ii = I + dt sum_j c_ij (-F_ij) x_ij x_ij^T.
__global__ void __launch_bounds__(kBlock) k_visc_precond(
    int64_t nf, const float4* __restrict__ x, const float* __restrict__ rho, const uint32_t* __restrict__ nlist,
    const uint32_t* __restrict__ ncnt, Kern kc, float dt, float mu, float2* __restrict__ Pinv) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float4 xi = x[i];
    const float eps2 = 0.01f * kc.h * kc.h;
    float b00 = 0.f, b01 = 0.f, b02 = 0.f, b11 = 0.f, b12 = 0.f, b22 = 0.f;
    for_each_nbr(nlist, nf, i, ncnt[i], [&](uint32_t j) {
        const float4 xj = x[j];
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float c = grad_factor(r2, kc) / (rho[j] * (r2 + eps2));
        b00 += c * dx * dx; b01 += c * dx * dy; b02 += c * dx * dz;
        b11 += c * dy * dy; b12 += c * dy * dz; b22 += c * dz * dz;
    });
    const float s = -dt * 10.0f * mu * kc.m / rho[i];
    const double a = 1.0 + (double)(s * b00), bq = (double)(s * b01), cq = (double)(s * b02);
    const double e = 1.0 + (double)(s * b11), f = (double)(s * b12), k2 = 1.0 + (double)(s * b22);
    const double A = e * k2 - f * f, B = -(bq * k2 - f * cq), C = bq * f - e * cq;
    const double det = a * A + bq * B + cq * C;
    const double id = 1.0 / det;
    // the block is symmetric, so is its inverse: its upper triangle
    // (00, 01, 02, 11, 12, 22) as three float2
    float2* o = Pinv + 3 * i;
    o[0] = make_float2((float)(A * id), (float)(B * id));
    o[1] = make_float2((float)(C * id), (float)((a * k2 - cq * cq) * id));
    o[2] = make_float2((float)(-(a * f - cq * bq) * id), (float)((a * e - bq * bq) * id));
}

// z = P r with P the symmetric inverse block stored as its upper triangle
__device__ __forceinline__ float4 apply3(const float2* P, float4 r) {
    const float2 p0 = P[0], p1 = P[1], p2 = P[2];   // (00, 01), (02, 11), (12, 22)
    float4 z;
    z.x = p0.x * r.x + p0.y * r.y + p1.x * r.z;
    z.y = p0.y * r.x + p1.y * r.y + p2.x * r.z;
    z.z = p1.x * r.x + p2.x * r.y + p2.y * r.z;
    z.w = 0.f;
    return z;
}

// FP64 sum of n partials part[k stride + off] in a fixed order, the same in
// every workgroup that calls it, returned to every thread of the workgroup.
__device__ double block_total(const double* __restrict__ part, int n, int stride, int off) {
    __shared__ double total;
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += kBlock) acc += part[(size_t)b * stride + off];
    acc = block_sum(acc);
    if (threadIdx.x == 0) total = acc;
    __syncthreads();
    const double t = total;
    __syncthreads();
    return t;
}

// CG start value: b = v + dt g and x0 = b + w dvisc, with dvisc the previous
// step's correction v* - b; both carry the volume m/rho (v.w) in w.
__global__ void k_cg_start(int64_t nf, const float4* __restrict__ v, const float4* __restrict__ dvisc,
                           float4* __restrict__ b, float4* __restrict__ x0, float dt, float gx, float gy, float gz,
                           float w) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float4 a = v[i];
    const float4 bb = make_float4(a.x + dt * gx, a.y + dt * gy, a.z + dt * gz, a.w);
    const float4 d = dvisc[i];
    b[i] = bb;
    x0[i] = make_float4(bb.x + w * d.x, bb.y + w * d.y, bb.z + w * d.z, a.w);
}

// The correction v* - b of the solve just finished (the next step's start).
__global__ void k_visc_correction(int64_t nf, const float4* __restrict__ vs, const float4* __restrict__ b,
                                  float4* __restrict__ dvisc) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float4 u = vs[i], bb = b[i];
    dvisc[i] = make_float4(u.x - bb.x, u.y - bb.y, u.z - bb.z, 0.f);
}

// Initial residual r = b - M x0, z = P r, p = z (w = m/rho), and the
// per-workgroup FP64 sums r.z, b.b, r.r (three per workgroup).
__global__ void k_cg_setup(int64_t nf, const float4* __restrict__ b, const float4* __restrict__ Mx,
                           const float2* __restrict__ Pinv, float4* __restrict__ r, float4* __restrict__ z,
                           float4* __restrict__ p, double* __restrict__ partials) {
    const int64_t i = particle_index();
    double rz = 0.0, bb2 = 0.0, rr = 0.0;
    if (i < nf) {
        const float4 bb = b[i], m = Mx[i];
        const float4 rv = make_float4(bb.x - m.x, bb.y - m.y, bb.z - m.z, bb.w);
        float4 zz = apply3(Pinv + 3 * i, rv);
        zz.w = bb.w;
        r[i] = rv;
        z[i] = zz;
        p[i] = zz;
        rz = (double)rv.x * zz.x + (double)rv.y * zz.y + (double)rv.z * zz.z;
        bb2 = (double)bb.x * bb.x + (double)bb.y * bb.y + (double)bb.z * bb.z;
        rr = (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z;
    }
    const double s0 = block_sum(rz);
    const double s1 = block_sum(bb2);
    const double s2 = block_sum(rr);
    if (threadIdx.x == 0) {
        partials[3 * (size_t)blockIdx.x] = s0;
        partials[3 * (size_t)blockIdx.x + 1] = s1;
        partials[3 * (size_t)blockIdx.x + 2] = s2;
    }
}

// The control block of iteration 0 from the set-up's sums (one workgroup).
__global__ void k_cg_init(const double* __restrict__ partials, int nblk, CgCtl* ctl, double tol, int32_t max_iters,
                          HostStatus* host) {
    const double rz = block_total(partials, nblk, 3, 0);
    const double bb = block_total(partials, nblk, 3, 1);
    const double rr = block_total(partials, nblk, 3, 2);
    if (threadIdx.x == 0) {
        CgCtl c{};
        c.rz = rz;
        c.rr = rr;
        c.bnorm = sqrt(bb);
        c.thresh = tol * c.bnorm;
        c.iters = 0;
        c.max_iters = max_iters;
        c.go = (sqrt(c.rr) > c.thresh && 0 < max_iters) ? 1 : 0;
        *ctl = c;
        host->cg = c;
    }
}

// One CG iteration is the mat-vec w = M u of the preconditioned residual u
// (with the per-workgroup sums of u.w) and this update, in the
// single-reduction form of preconditioned CG (Chronopoulos and Gear): with
// gamma = r.u and delta = u.w,
//   beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev)
//   (first iteration: beta = 0, alpha = gamma / delta),
//   p = u + beta p,  s = w + beta s  (s = M p),  x += alpha p,  r -= alpha s,
//   u = P r,  and the per-workgroup sums r.u, r.r for the next iteration.
// The iteration reads the control block `ctl` and workgroup 0 writes the
// next one into the other slot of a pair, so no launch writes a block it
// reads.  The stop rule (|r| <= tol |b|, or max_iters) is evaluated at the
// start of the next update from its predecessor's sums (the first update
// takes the set-up's decision); a stopped block is carried forward.
__global__ void k_cg_update(int64_t nf, float4* __restrict__ xv, float4* __restrict__ r, float4* __restrict__ u,
                            float4* __restrict__ p, float4* __restrict__ sv, const float4* __restrict__ w,
                            const float2* __restrict__ Pinv, const CgCtl* ctl, CgCtl* next,
                            const double* __restrict__ prev_part, int nprev, const double* __restrict__ uw_part,
                            int nuw, double* __restrict__ partials, HostStatus* host, bool first) {
    CgCtl c = *ctl;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!c.go) {
        if (lead) {
            *next = c;
            host->cg = c;
        }
        return;
    }
    // the particle's vectors are loaded first, the three sums (gamma and r.r
    // of the previous update, delta of the mat-vec) then formed in one pass
    // and one workgroup reduction, in the same order in every workgroup
    const int64_t i = particle_index();
    const bool live = i < nf;
    float4 uu{}, ww{}, pp{}, ss{}, xx{}, rv{};
    float2 P[3];
    if (live) {
        uu = u[i];
        ww = w[i];
        if (!first) {
            pp = p[i];
            ss = sv[i];
        }
        xx = xv[i];
        rv = r[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) P[k] = Pinv[3 * i + k];
    }
    double sg = 0.0, sr = 0.0, sd = 0.0;
    if (!first)
        for (int b = threadIdx.x; b < nprev; b += kBlock) {
            sg += prev_part[2 * (size_t)b];
            sr += prev_part[2 * (size_t)b + 1];
        }
    for (int b = threadIdx.x; b < nuw; b += kBlock) sd += uw_part[b];
    {
        __shared__ double ws[3][kBlock / 64];
        __shared__ double tot[3];
        sg = wave_sum(sg);
        sr = wave_sum(sr);
        sd = wave_sum(sd);
        if ((threadIdx.x & 63) == 0) {
            ws[0][threadIdx.x >> 6] = sg;
            ws[1][threadIdx.x >> 6] = sr;
            ws[2][threadIdx.x >> 6] = sd;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double t = ws[threadIdx.x][0];
            for (int k = 1; k < kBlock / 64; ++k) t += ws[threadIdx.x][k];
            tot[threadIdx.x] = t;
        }
        __syncthreads();
        sg = tot[0];
        sr = tot[1];
        sd = tot[2];
    }
    double gamma = c.rz, rr = c.rr;
    if (!first) {
        gamma = sg;
        rr = sr;
        if (!(sqrt(rr) > c.thresh && c.iters < c.max_iters)) {
            c.go = 0;
            c.rr = rr;
            c.rz = gamma;
            if (lead) {
                *next = c;
                host->cg = c;
            }
            return;
        }
    }
    const double delta = sd;
    const double beta = first ? 0.0 : gamma / c.rz;
    const double alpha = first ? gamma / delta : gamma / (delta - beta * gamma / c.alpha);
    const float a = (float)alpha, bt = (float)beta;
    double ru = 0.0, r2 = 0.0;
    if (live) {
        if (first) {
            pp = uu;
            ss = ww;
        } else {
            pp.x = uu.x + bt * pp.x; pp.y = uu.y + bt * pp.y; pp.z = uu.z + bt * pp.z;
            ss.x = ww.x + bt * ss.x; ss.y = ww.y + bt * ss.y; ss.z = ww.z + bt * ss.z;
        }
        p[i] = pp;
        sv[i] = ss;
        xx.x += a * pp.x; xx.y += a * pp.y; xx.z += a * pp.z;
        rv.x -= a * ss.x; rv.y -= a * ss.y; rv.z -= a * ss.z;
        xv[i] = xx;
        r[i] = rv;
        float4 zz = apply3(P, rv);
        zz.w = rv.w;
        u[i] = zz;
        ru = (double)rv.x * zz.x + (double)rv.y * zz.y + (double)rv.z * zz.z;
        r2 = (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z;
    }
    const double s0 = block_sum(ru);
    const double s1 = block_sum(r2);
    if (threadIdx.x == 0) {
        partials[2 * (size_t)blockIdx.x] = s0;
        partials[2 * (size_t)blockIdx.x + 1] = s1;
    }
    if (lead) {
        c.rz = gamma;
        c.rr = rr;
        c.alpha = alpha;
        c.beta = beta;
        c.iters += 1;
        *next = c;
        host->cg = c;
    }
}

__global__ void k_warm_setup(int64_t nf, float4* __restrict__ x, const float* __restrict__ rho,
                             float* __restrict__ K, float* __restrict__ kappa, float warm_factor,
                             float* __restrict__ Ksave) {
    const int64_t i = particle_index();
    if (i >= nf) return;
    const float Ki = K[i];
    if (Ksave) Ksave[i] = Ki;
    const float k0 = warm_factor * Ki;
    kappa[i] = k0;
    K[i] = 0.0f;
    x[i].w = k0 / rho[i];
}

}  // namespace

// ================================================================== launchers
// lanes per particle of the neighbour sums (measured at 1.23M particles)
constexpr int kLanesDensity = 2, kLanesPressure = 2, kLanesPredict = 2, kLanesXsph = 4;
constexpr int kLanesXsphPress = 2;   // the non-pressure pass that also applies a pressure or takes the check

#define LAUNCH(kern, n, ...)                                                        \
    do {                                                                            \
        hipLaunchKernelGGL(kern, dim3(grid_blocks(n)), dim3(kBlock), 0, s, __VA_ARGS__); \
        return hipGetLastError();                                                   \
    } while (0)

static inline uint32_t plain_blocks(int64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(plain_blocks(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(plain_blocks(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_keys_hist(const float4* x, int64_t n, Grid g, uint32_t* key, uint32_t* slot, uint32_t* count,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    LAUNCH(k_keys_hist, n, x, n, g, key, slot, count);
}

// partials needs ceil(n / 4096) + 2 + ceil(ceil(n/4096)/4096) entries.
hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* partials, hipStream_t s) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles > kScanTile) return hipErrorInvalidValue;   // > 16.7M cells
    uint32_t* tile_sum = partials;               // [tiles]
    uint32_t* tile_base = partials + tiles;      // [tiles]
    uint32_t* total = partials + 2 * tiles;      // [1]
    hipLaunchKernelGGL(k_scan_local, dim3((uint32_t)tiles), dim3(kBlock), 0, s, in, n, out, tile_sum);
    hipLaunchKernelGGL(k_scan_local, dim3(1), dim3(kBlock), 0, s, tile_sum, tiles, tile_base, total);
    hipLaunchKernelGGL(k_scan_add, dim3(plain_blocks(n + 1)), dim3(kBlock), 0, s, out, n, tile_base, total);
    return hipGetLastError();
}

hipError_t launch_scatter(const uint32_t* key, const uint32_t* slot, const uint32_t* start, int64_t n, uint32_t* src,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    LAUNCH(k_scatter, n, key, slot, start, n, src);
}

hipError_t launch_cell_sort(const uint32_t* start, int64_t ncell, uint32_t* src, const int32_t* id, uint32_t* flags,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_cell_sort, dim3(plain_blocks(ncell)), dim3(kBlock), 0, s, start, ncell, src, id, flags);
    return hipGetLastError();
}

hipError_t launch_gather_fluid(const uint32_t* src, int64_t n, const float4* x, const float4* v, const float* K,
                               const float* Kv, const float* rho, const int32_t* id, const float4* dv, float4* xo,
                               float4* vo, float* Ko, float* Kvo, float* rhoo, int32_t* ido, float4* dvo,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    LAUNCH(k_gather_fluid, n, src, n, x, v, K, Kv, rho, id, dv, xo, vo, Ko, Kvo, rhoo, ido, dvo);
}

hipError_t launch_gather_boundary(const uint32_t* src, int64_t n, const float4* x, const float4* v, const int32_t* id,
                                  float4* xo, float4* vo, int32_t* ido, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    LAUNCH(k_gather_boundary, n, src, n, x, v, id, xo, vo, ido);
}

hipError_t launch_nbr_build(const float4* x, int64_t nf, const float4* xb, const uint32_t* start_f,
                            const uint32_t* start_b, Grid g, uint32_t* nlist, uint32_t* ncnt, int32_t capf,
                            uint32_t* blist, uint32_t* bcnt, int32_t capb, uint32_t* flags,
                            unsigned long long* partials, HostStatus* host, hipStream_t s) {
    const uint32_t nblk = grid_blocks(nf);
    hipLaunchKernelGGL(k_nbr_build, dim3(nblk), dim3(kBlock), 0, s, x, nf, xb, start_f, start_b, g, nlist, ncnt,
                       capf, blist, bcnt, capb, flags, partials);
    hipLaunchKernelGGL(k_finish_nstats, dim3(1), dim3(kBlock), 0, s, partials, (int)nblk, (const uint32_t*)flags,
                       host);
    return hipGetLastError();
}

hipError_t launch_boundary_psi(float4* xb, int64_t nb, const uint32_t* start_b, Grid g, Kern kc, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    LAUNCH(k_boundary_psi, nb, xb, nb, start_b, g, kc);
}

hipError_t launch_max_v2(const float4* v, int64_t n, uint32_t* partials, HostStatus* host, hipStream_t s) {
    const uint32_t nblk = grid_blocks(n);
    hipLaunchKernelGGL(k_max_v2, dim3(nblk), dim3(kBlock), 0, s, v, n, partials);
    hipLaunchKernelGGL(k_finish_max_u32, dim3(1), dim3(kBlock), 0, s, partials, (int)nblk, host,
                       (const int32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_density_alpha(int64_t nf, float4* x, const float4* v, float4* vout, const uint32_t* nlist,
                                const uint32_t* ncnt, const float4* xb, const float4* vb, const uint32_t* blist,
                                const uint32_t* bcnt, Kern kc, float* rho, float* alpha, float4* v_in, float* Kv,
                                float dt, float warm_factor, float pci_c, float* din, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    if (din && vout == v) return hipErrorInvalidValue;   // neighbours read v while the pass writes
    const dim3 grid(grid_blocks(kLanesDensity * nf)), block(kBlock);
#define DENSITY_LAUNCH(W, D)                                                                                      \
    hipLaunchKernelGGL((k_density_alpha<kLanesDensity, W, D>), grid, block, 0, s, nf, x, v, vout, nlist, ncnt, xb, \
                       vb, blist, bcnt, kc, rho, alpha, v_in, Kv, dt, warm_factor, pci_c, din)
    if (warm_factor > 0.0f) {
        if (din) DENSITY_LAUNCH(true, true);
        else DENSITY_LAUNCH(true, false);
    } else {
        if (din) DENSITY_LAUNCH(false, true);
        else DENSITY_LAUNCH(false, false);
    }
#undef DENSITY_LAUNCH
    return hipGetLastError();
}

hipError_t launch_pressure_update(int64_t nf, const float4* x, float4* v, const float* kappa, float* Kacc,
                                  float* kappa_last, const uint32_t* nlist, const uint32_t* ncnt, const float4* xb,
                                  const uint32_t* blist, const uint32_t* bcnt, Kern kc, float dt, const int32_t* go,
                                  hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_pressure_update<kLanesPressure>, kLanesPressure * nf, nf, x, v, kappa, Kacc, kappa_last, nlist, ncnt, xb, blist, bcnt, kc, dt,
           go);
}

hipError_t launch_predict(int mode, int64_t nf, float4* x, const float4* v, const float* rho, const float* alpha,
                          float* kappa, const uint32_t* nlist, const uint32_t* ncnt, const float4* xb,
                          const float4* vb, const uint32_t* blist, const uint32_t* bcnt, Kern kc, float dt,
                          double* partials, SolveCtl* ctl, bool first, float* dout, int* nparts,
                          hipStream_t s) {
    const uint32_t nblk = grid_blocks(kLanesPredict * nf);
    *nparts = nf > 0 ? (int)nblk : 0;
    if (nf <= 0) return hipSuccess;
    const int32_t* go = first ? nullptr : &ctl->go;
    if (mode == 0)
        hipLaunchKernelGGL((k_predict<0, kLanesPredict>), dim3(nblk), dim3(kBlock), 0, s, nf, x, v, rho, alpha, kappa, nlist, ncnt, xb,
                           vb, blist, bcnt, kc, dt, partials, go, dout);
    else
        hipLaunchKernelGGL((k_predict<1, kLanesPredict>), dim3(nblk), dim3(kBlock), 0, s, nf, x, v, rho, alpha, kappa, nlist, ncnt, xb,
                           vb, blist, bcnt, kc, dt, partials, go, nullptr);
    return hipGetLastError();
}

hipError_t launch_eos(int64_t nf, float4* x, const float* rho, float* kappa, float* K, Kern kc, float k, float gamma,
                      double* partials, int* nparts, hipStream_t s) {
    const uint32_t nblk = grid_blocks(nf);
    *nparts = nf > 0 ? (int)nblk : 0;
    if (nf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eos, dim3(nblk), dim3(kBlock), 0, s, nf, x, rho, kappa, K, kc, k, gamma, partials);
    return hipGetLastError();
}

hipError_t launch_solve_finish(const double* partials, int nblk, SolveCtl* ctl, bool first, const SolveCtl& init,
                               HostStatus* host, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_solve, dim3(1), dim3(kFinishThreads), 0, s, partials, nblk, ctl, first, init, host);
    return hipGetLastError();
}

hipError_t launch_nonpressure(int model, int64_t nf, float4* x, const float4* v, float4* vout, const float* rho,
                              const uint32_t* nlist, const uint32_t* ncnt, Kern kc, float dt, float gx, float gy,
                              float gz, float visc, float* K, float* kappa, float warm_factor, bool setup_warm,
                              bool press, const float4* xb, const uint32_t* blist, const uint32_t* bcnt,
                              float* kappa_last, const DivCheck* div, int* nparts, hipStream_t s) {
    if (nparts) *nparts = 0;
    if (nf <= 0) return hipSuccess;
    const dim3 block(kBlock);
    const DivCheck dc = div ? *div : DivCheck{};
#define NONPRESSURE(M, P, D)                                                                                      \
    do {                                                                                                          \
        constexpr int lanes = (M == 0 && !P && !D) ? 1 : ((P || D) ? kLanesXsphPress : kLanesXsph);               \
        const uint32_t nblk = grid_blocks(lanes * nf);                                                            \
        if (nparts) *nparts = (int)nblk;                                                                          \
        hipLaunchKernelGGL((k_nonpressure<M, lanes, P, D>), dim3(nblk), block, 0, s, nf, x, v, vout, rho, nlist,  \
                           ncnt, kc, dt, gx, gy, gz, visc, K, kappa, warm_factor, setup_warm, xb, blist, bcnt,    \
                           kappa_last, dc);                                                                       \
    } while (0)
#define NONPRESSURE_M(M)                                       \
    do {                                                       \
        if (press) {                                           \
            if (div) NONPRESSURE(M, true, true);               \
            else NONPRESSURE(M, true, false);                  \
        } else {                                               \
            if (div) NONPRESSURE(M, false, true);              \
            else NONPRESSURE(M, false, false);                 \
        }                                                      \
    } while (0)
    // model 0 without pressure or check: gravity only, one lane per particle
    if (model == 1) NONPRESSURE_M(1);
    else if (model == 2) NONPRESSURE_M(2);
    else NONPRESSURE_M(0);
#undef NONPRESSURE_M
#undef NONPRESSURE
    return hipGetLastError();
}

hipError_t launch_div_resume(int64_t nf, float4* x, float* kappa, float* K, const float2* kvs, const float* Ksaved,
                             hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_div_resume, nf, nf, x, kappa, K, kvs, Ksaved);
}

hipError_t launch_features(int64_t nf, const float* rho, const float* alpha, const float* K, const uint32_t* ncnt,
                           const uint32_t* bcnt, const float* d, Kern kc, float dt, float alpha_ref, float* feat,
                           hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_features, nf, nf, rho, alpha, K, ncnt, bcnt, d, kc, dt, alpha_ref, feat);
}
hipError_t launch_warm_learned(int64_t nf, float4* x, const float* rho, const float* alpha, const float* y, float* K,
                               float* kappa, float dt, float rho0, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_warm_learned, nf, nf, x, rho, alpha, y, K, kappa, dt, rho0);
}

hipError_t launch_trace_target(int64_t nf, const float* alpha, const float* K, float dt, float rho0, float* target,
                               hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_trace_target, nf, nf, alpha, K, dt, rho0, target);
}

hipError_t launch_warm_setup(int64_t nf, float4* x, const float* rho, float* K, float* kappa, float warm_factor,
                             float* Ksave, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_warm_setup, nf, nf, x, rho, K, kappa, warm_factor, Ksave);
}

hipError_t launch_integrate(int64_t nf, float4* x, const float4* v, float dt, uint32_t* partials, HostStatus* host,
                            const int32_t* gate, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    const uint32_t nblk = grid_blocks(nf);
    hipLaunchKernelGGL(k_integrate, dim3(nblk), dim3(kBlock), 0, s, nf, x, v, dt, partials, gate);
    if (partials)
        hipLaunchKernelGGL(k_finish_max_u32, dim3(1), dim3(kBlock), 0, s, partials, (int)nblk, host, gate);
    return hipGetLastError();
}

hipError_t launch_rigid_force(int64_t nf, const float4* x, const float* rho, const float* K, const float* Kv,
                              const uint32_t* blist, const uint32_t* bcnt, const float4* xb, const float4* vb,
                              Kern kc, int32_t nbody, const double* com, double* partials, HostStatus* host,
                              hipStream_t s) {
    const uint32_t nblk = grid_blocks(nf);
    hipLaunchKernelGGL(k_rigid_force, dim3(nblk), dim3(kBlock), 0, s, nf, x, rho, K, Kv, blist, bcnt, xb, vb, kc,
                       nbody, com, partials, 0.0f, nullptr);
    hipLaunchKernelGGL(k_finish_rigid, dim3(6 * nbody), dim3(kBlock), 0, s, partials, (int)nblk, host);
    return hipGetLastError();
}

hipError_t launch_rigid_boundary(int64_t nb, float4* xb, float4* vb, const int32_t* bid, const double* local,
                                 const BodyPose* poses, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    LAUNCH(k_rigid_boundary, nb, nb, xb, vb, bid, local, poses, nullptr);
}

// Strong coupling: the pass's reaction per body (fixed-order sums of the
// workgroup partials, one workgroup per output), then one thread per body
// advances its velocity and the step's totals.
__global__ void k_rigid_pass_finish(const double* __restrict__ partials, int nblk, double* __restrict__ ft,
                                    const int32_t* __restrict__ go) {
    if (go != nullptr && *go == 0) return;
    const int o = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) acc += partials[(size_t)o * nblk + b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) ft[o] = acc;
}

__global__ void k_rigid_pass_update(int32_t nbody, const double* __restrict__ ft, const BodyDyn* __restrict__ dyn,
                                    BodyPose* __restrict__ poses, double* __restrict__ total, float dt,
                                    const int32_t* __restrict__ go, HostStatus* host) {
#pragma clang fp contract(off)
    if (go != nullptr && *go == 0) return;
    const int b = threadIdx.x;
    if (b >= nbody) return;
    const double* F = ft + 6 * b;
    const BodyDyn& D = dyn[b];
    BodyPose& P = poses[b];
    const double h = (double)dt;
    for (int a = 0; a < 3; ++a) {
        P.vel[a] += h * F[a] / D.mass;
        P.omega[a] += h * (D.Iwinv[3 * a] * F[3] + D.Iwinv[3 * a + 1] * F[4] + D.Iwinv[3 * a + 2] * F[5]);
    }
    for (int a = 0; a < 6; ++a) {
        total[6 * b + a] += F[a];
        host->rigid[6 * b + a] = total[6 * b + a];
    }
}

__global__ void k_rigid_gravity(int32_t nbody, const BodyDyn* __restrict__ dyn, BodyPose* __restrict__ poses,
                                double gx, double gy, double gz, float dt) {
#pragma clang fp contract(off)
    const int b = threadIdx.x;
    if (b >= nbody) return;
    const BodyDyn& D = dyn[b];
    BodyPose& P = poses[b];
    const double h = (double)dt, g[3] = {gx, gy, gz};
    double L[3], gy3[3];
    for (int a = 0; a < 3; ++a) L[a] = D.Iw[3 * a] * P.omega[0] + D.Iw[3 * a + 1] * P.omega[1] + D.Iw[3 * a + 2] * P.omega[2];
    gy3[0] = P.omega[1] * L[2] - P.omega[2] * L[1];
    gy3[1] = P.omega[2] * L[0] - P.omega[0] * L[2];
    gy3[2] = P.omega[0] * L[1] - P.omega[1] * L[0];
    double dw[3];
    for (int a = 0; a < 3; ++a) dw[a] = D.Iwinv[3 * a] * gy3[0] + D.Iwinv[3 * a + 1] * gy3[1] + D.Iwinv[3 * a + 2] * gy3[2];
    for (int a = 0; a < 3; ++a) {
        P.vel[a] += h * g[a];
        P.omega[a] -= h * dw[a];
    }
}

hipError_t launch_rigid_couple(int64_t nf, const float4* x, const uint32_t* blist, const uint32_t* bcnt,
                               float4* xb, float4* vb, const int32_t* bid, const double* local, Kern kc,
                               int32_t nbody, const double* com, int64_t nb, double* partials, float xw_scale,
                               float dt, const int32_t* go, const BodyDyn* dyn, BodyPose* poses, double* ft_total,
                               HostStatus* host, hipStream_t s) {
    if (nbody <= 0) return hipSuccess;
    const uint32_t nblk = grid_blocks(nf);
    double* ft = ft_total + 6 * kMaxBodies;   // this pass's reaction, after the totals
    hipLaunchKernelGGL(k_rigid_force, dim3(nblk), dim3(kBlock), 0, s, nf, x, nullptr, nullptr, nullptr, blist, bcnt,
                       xb, vb, kc, nbody, com, partials, xw_scale, go);
    hipLaunchKernelGGL(k_rigid_pass_finish, dim3(6 * nbody), dim3(kBlock), 0, s, partials, (int)nblk, ft, go);
    hipLaunchKernelGGL(k_rigid_pass_update, dim3(1), dim3(64), 0, s, nbody, ft, dyn, poses, ft_total, dt, go, host);
    if (nb > 0)
        hipLaunchKernelGGL(k_rigid_boundary, dim3(grid_blocks(nb)), dim3(kBlock), 0, s, nb, xb, vb, bid, local,
                           poses, go);
    return hipGetLastError();
}

hipError_t launch_rigid_gravity(int32_t nbody, int64_t nb, float4* xb, float4* vb, const int32_t* bid,
                                const double* local, const BodyDyn* dyn, BodyPose* poses, double gx, double gy,
                                double gz, float dt, hipStream_t s) {
    if (nbody <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rigid_gravity, dim3(1), dim3(64), 0, s, nbody, dyn, poses, gx, gy, gz, dt);
    if (nb > 0)
        hipLaunchKernelGGL(k_rigid_boundary, dim3(grid_blocks(nb)), dim3(kBlock), 0, s, nb, xb, vb, bid, local,
                           poses, nullptr);
    return hipGetLastError();
}

hipError_t launch_visc_precond(int64_t nf, const float4* x, const float* rho, const uint32_t* nlist,
                               const uint32_t* ncnt, Kern kc, float dt, float mu, float2* Pinv, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_visc_precond, nf, nf, x, rho, nlist, ncnt, kc, dt, mu, Pinv);
}

constexpr int kLanesVisc = 2;

int visc_matvec_parts(int64_t nf) { return (int)grid_blocks(kLanesVisc * nf); }

hipError_t launch_visc_matvec(int64_t nf, const float4* x, const float4* p, float4* Mp, const uint32_t* nlist,
                              const uint32_t* ncnt, Kern kc, float dt, float mu, const int32_t* go,
                              double* partials, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_visc_matvec<kLanesVisc>, kLanesVisc * nf, nf, x, p, Mp, nlist, ncnt, kc, dt, mu, go, partials);
}

hipError_t launch_cg_start(int64_t nf, const float4* v, const float4* dvisc, float4* b, float4* x0, float dt,
                           float gx, float gy, float gz, float w, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_cg_start, nf, nf, v, dvisc, b, x0, dt, gx, gy, gz, w);
}

hipError_t launch_visc_correction(int64_t nf, const float4* vs, const float4* b, float4* dvisc, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    LAUNCH(k_visc_correction, nf, nf, vs, b, dvisc);
}

hipError_t launch_cg_setup(int64_t nf, const float4* b, const float4* Mx, const float2* Pinv, float4* r, float4* z,
                           float4* p, double* partials, CgCtl* ctl, double tol, int32_t max_iters,
                           HostStatus* host, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    const uint32_t nblk = grid_blocks(nf);
    hipLaunchKernelGGL(k_cg_setup, dim3(nblk), dim3(kBlock), 0, s, nf, b, Mx, Pinv, r, z, p, partials);
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kBlock), 0, s, (const double*)partials, (int)nblk, ctl, tol,
                       max_iters, host);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(int64_t nf, float4* xv, float4* r, float4* u, float4* p, float4* sv, const float4* w,
                               const float2* Pinv, const CgCtl* ctl, CgCtl* next, const double* prev_part,
                               const double* uw_part, int nuw, double* partials, HostStatus* host, bool first,
                               hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    const uint32_t nblk = grid_blocks(nf);
    hipLaunchKernelGGL(k_cg_update, dim3(nblk), dim3(kBlock), 0, s, nf, xv, r, u, p, sv, w, Pinv, ctl, next, prev_part,
                       (int)nblk, uw_part, nuw, partials, host, first);
    return hipGetLastError();
}

uint32_t reduction_blocks(int64_t n) { return grid_blocks(n); }

}  // namespace sph
