// sph_device.h -- device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "sph_internal.h"

namespace sph {
namespace {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ uint32_t logical_block() {
    const uint32_t b = blockIdx.x, per = gridDim.x >> 3;
    return (b & 7u) * per + (b >> 3);
}

__device__ __forceinline__ int64_t particle_index() {
    return (int64_t)logical_block() * kBlock + threadIdx.x;
}

inline uint32_t grid_blocks(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (uint32_t)((b + 7) & ~int64_t(7));   // a multiple of the 8 XCDs
}

// Cell coordinate: clamp(floor(fl32(fl32(x - o) * inv)), 0, n - 1); NaN -> 0.
__device__ __forceinline__ int32_t cell_coord(float x, float o, float inv, int32_t n) {
#pragma clang fp contract(off)
    const float t = (x - o) * inv;
    const float f = floorf(t);
    if (!(f >= 0.0f)) return 0;
    if (f > (float)(n - 1)) return n - 1;
    return (int32_t)f;
}

__device__ __forceinline__ uint32_t cell_key(const Grid& g, float4 p) {
    const int32_t cx = cell_coord(p.x, g.o[0], g.inv, g.n[0]);
    const int32_t cy = cell_coord(p.y, g.o[1], g.inv, g.n[1]);
    const int32_t cz = cell_coord(p.z, g.o[2], g.inv, g.n[2]);
    return (uint32_t)(cx + g.n[0] * (cy + g.n[1] * cz));
}

// FP32 squared distance ((dx*dx + dy*dy) + dz*dz), no FMA: the neighbour predicate.
__device__ __forceinline__ float dist2_exact(float4 a, float4 b) {
#pragma clang fp contract(off)
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float s = xx + yy;
    return s + zz;
}

// Cubic spline (support h): grad_i W(x_ij) = grad_factor * x_ij.  Branch-free
// (coincident particles select 0) so that neighbour loops can issue their
// gathers ahead of the arithmetic; v_rsq_f32 directly (r^2 is never denormal
// for distinct particles).
__device__ __forceinline__ float inv_dist(float r2) { return r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f; }

__device__ __forceinline__ float grad_factor(float r2, const Kern& kc) {
    const float rinv = inv_dist(r2);
    const float q = r2 * rinv * kc.inv_h;
    const float t = fmaxf(1.0f - q, 0.0f);
    const float fp = q <= 0.5f ? q * (3.0f * q - 2.0f) : -t * t;
    return kc.kg * fp * rinv;
}

__device__ __forceinline__ float kernel_W(float r2, const Kern& kc) {
    const float q = r2 * inv_dist(r2) * kc.inv_h;
    const float t = fmaxf(1.0f - q, 0.0f);
    return q <= 0.5f ? kc.k * (6.0f * q * q * (q - 1.0f) + 1.0f) : kc.k * 2.0f * t * t * t;
}

// Neighbour lists (32-bit sorted indices): entry k of particle i sits in
// chunk k/4 of four entries, chunks stored chunk-major,
// list[4 ((k/4) nf + i) + k%4]; a wave reads or writes one chunk of its 64
// consecutive particles as a single coalesced 1 KB access.
__device__ __forceinline__ int64_t list_index(int64_t nf, int64_t i, uint32_t k) {
    return (((int64_t)(k >> 2) * nf + i) << 2) + (k & 3u);
}

// Visit the first n entries of particle i's list: one 16-byte load brings
// four entries, and the four gathers done by `f` are issued before any of the
// arithmetic, so each wave keeps several gathers in flight.
template <class F>
__device__ __forceinline__ void for_each_nbr(const uint32_t* __restrict__ list, int64_t nf, int64_t i, uint32_t n,
                                             F&& f) {
    const uint4* p = reinterpret_cast<const uint4*>(list) + i;
    uint32_t k = 0;
    for (; k + 4 <= n; k += 4) {
        const uint4 q = *p;
        p += nf;
        f(q.x);
        f(q.y);
        f(q.z);
        f(q.w);
    }
    if (k < n) {   // the last chunk is allocated whole; entries past n are not used
        const uint4 q = *p;
        f(q.x);
        if (k + 1 < n) f(q.y);
        if (k + 2 < n) f(q.z);
    }
}

// A particle's term of a solver error: its clamped (compression-only)
// deviation, except that a non-finite deviation passes through unclamped
// (fmaxf would turn NaN into 0), so that a non-finite state makes the
// error non-finite and the host reports it instead of declaring convergence.
__device__ __forceinline__ double err_term(float dev, float clamped) {
    return (double)(__builtin_isfinite(dev) ? clamped : dev);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block-wide FP64 sum in a fixed order; the result is valid in thread 0.
__device__ double block_sum(double v) {
    __shared__ double ws[kBlock / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = ws[0];
        for (int w = 1; w < kBlock / 64; ++w) r += ws[w];
    }
    __syncthreads();
    return r;
}

// Reductions are two-phase: every workgroup stores its partial with a plain
// store, and a one-workgroup finishing kernel sums the partials in workgroup
// order.  The kernel boundary orders the two phases; no device-scope fence or
// atomic is needed (an agent-scope fence on the multi-XCD part writes back the
// XCD's L2, which costs far more than one extra launch).
//
// The rigid force and torque into the host status: workgroup o sums output
// o's partials in workgroup order, stored output-major (partials[o nblk + b])
__global__ void k_finish_rigid(const double* __restrict__ partials, int nblk, HostStatus* host) {
    const int o = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) acc += partials[(size_t)o * nblk + b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) host->rigid[o] = acc;
}

// FP64 sum over a workgroup of NT threads in a fixed order; valid in thread 0.
template <int NT>
__device__ double block_sum_n(double v) {
    __shared__ double ws[NT / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = ws[0];
        for (int w = 1; w < NT / 64; ++w) r += ws[w];
    }
    __syncthreads();
    return r;
}

// Workgroup maximum of kBlock threads (exact in any order); valid in thread 0.
__device__ float block_max(float v) {
    __shared__ float wm[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_down(v, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = 0.0f;
    if (threadIdx.x == 0) {
        r = wm[0];
        for (int w = 1; w < kBlock / 64; ++w) r = fmaxf(r, wm[w]);
    }
    __syncthreads();
    return r;
}

template <int NT>
__device__ double block_max_n(double v) {
    __shared__ double wm[NT / 64];
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = wm[0];
        for (int w = 1; w < NT / 64; ++w) r = fmax(r, wm[w]);
    }
    __syncthreads();
    return r;
}

constexpr int kFinishThreads = 1024;   // the solve finish sums ~10^4 partials per pass

// Finish of a predict pass: err = scale * (sum of the partials in a fixed
// order); the solve's first finish starts the control block from init, a
// later one counts the iteration; then decide whether another one is due:
// exactly `forced` iterations, else while err > eta (or, with eta_max > 0,
// err_max > eta_max, err_max from the per-workgroup maxima stored after the
// sums) and fewer than max_iters.  Nothing happens once go is 0.  The block
// is mirrored to host.
__global__ void __launch_bounds__(kFinishThreads) k_finish_solve(const double* __restrict__ partials, int nblk,
                                                                 SolveCtl* ctl, bool first, SolveCtl init,
                                                                 HostStatus* host) {
    if (!first && ctl->go == 0) return;
    const bool with_max = (first ? init.eta_max : ctl->eta_max) > 0.0;
    double acc = 0.0, mx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kFinishThreads) {
        acc += partials[b];
        if (with_max) mx = fmax(mx, partials[nblk + b]);
    }
    acc = block_sum_n<kFinishThreads>(acc);
    if (with_max) mx = block_max_n<kFinishThreads>(mx);
    if (threadIdx.x == 0) {
        SolveCtl c = first ? init : *ctl;
        if (first) c.iters = 0;
        else c.iters += 1;
        c.err = acc * c.scale;
        c.err_max = with_max ? mx * c.max_scale : 0.0;
        const bool above = c.err > c.eta || (with_max && c.err_max > c.eta_max);
        c.go = c.forced >= 0 ? (c.iters < c.forced ? 1 : 0) : ((above && c.iters < c.max_iters) ? 1 : 0);
        *ctl = c;
        host->solve = c;
    }
}

// neighbour statistics per workgroup (kNStats fields): min, max, then sums
// Also mirrors the build flags to host.
__global__ void k_finish_nstats(const unsigned long long* __restrict__ partials, int nblk,
                                const uint32_t* __restrict__ flags, HostStatus* host) {
    // per lane over the partials, then across the wave with shuffles, then
    // across the workgroup's waves (integers: the order does not matter)
    unsigned long long a[kNStats];
    a[0] = ~0ull;
    for (int f = 1; f < kNStats; ++f) a[f] = 0ull;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        const unsigned long long* p = partials + (size_t)kNStats * b;
        a[0] = min(a[0], p[0]);
        a[1] = max(a[1], p[1]);
        for (int f = 2; f < kNStats; ++f) a[f] += p[f];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a[0] = min(a[0], (unsigned long long)__shfl_xor(a[0], off, 64));
        a[1] = max(a[1], (unsigned long long)__shfl_xor(a[1], off, 64));
        for (int f = 2; f < kNStats; ++f) a[f] += __shfl_xor(a[f], off, 64);
    }
    __shared__ unsigned long long s[kNStats][kBlock / 64];
    if ((threadIdx.x & 63) == 0)
        for (int f = 0; f < kNStats; ++f) s[f][threadIdx.x >> 6] = a[f];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            a[0] = min(a[0], s[0][w]);
            a[1] = max(a[1], s[1][w]);
            for (int f = 2; f < kNStats; ++f) a[f] += s[f][w];
        }
        for (int f = 0; f < kNStats; ++f) host->nstats[f] = a[f];
        host->flags = *flags;
    }
}

// gate (nullable): nothing happens while *gate != 0
__global__ void k_finish_max_u32(const uint32_t* __restrict__ partials, int nblk, HostStatus* host,
                                 const int32_t* __restrict__ gate) {
    if (gate != nullptr && *gate != 0) return;
    uint32_t m = 0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) m = max(m, partials[b]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
    __shared__ uint32_t s[kBlock / 64];
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = max(m, s[w]);
        host->vmax_bits = m;
    }
}


// Append the candidates c in [b, e) (ascending) with c != skip and the FP32
// predicate d^2 < h^2 to particle i's list.  A range is tested 32 candidates
// at a time into a bit mask (four candidates' loads issued ahead of the
// tests; one to three for the tail), then the set bits are appended in
// ascending order: the per-candidate work is the distance and one bit, the
// list bookkeeping runs once per accepted neighbour.  Accepted entries shift
// into buf (oldest in buf.x) and go out as whole 16-byte chunks; list_flush
// stores the last, partial one.  chunk points at the particle's next chunk
// (list chunk cnt/4 of particle i) and steps by nf chunks per store.  cnt
// counts every neighbour, entries past cap are dropped (the caller flags the
// overflow).  SKIP: the range may hold the particle itself.
__device__ __forceinline__ void append_mask(uint32_t mask, uint32_t base, uint4*& chunk, int64_t nf, int32_t cap,
                                            uint32_t& cnt, uint4& buf) {
    while (mask) {
        const uint32_t j = (uint32_t)__builtin_ctz(mask);
        mask &= mask - 1u;
        if (cnt < (uint32_t)cap) {
            buf.x = buf.y;
            buf.y = buf.z;
            buf.z = buf.w;
            buf.w = base + j;
            if ((cnt & 3u) == 3u) {
                *chunk = buf;
                chunk += nf;
            }
        }
        ++cnt;
    }
}

template <bool SKIP, typename Load>
__device__ __forceinline__ void scan_with(Load load, uint32_t b, uint32_t e, float4 xi, uint32_t skip, float h2,
                                          uint4*& chunk, int64_t nf, int32_t cap, uint32_t& cnt, uint4& buf) {
    for (uint32_t base = b; base < e; base += 32u) {
        const uint32_t n = min(e - base, 32u);
        auto q = [&](uint32_t k) { return load(base + k); };
        uint32_t mask = 0u;
        auto test = [&](uint32_t k, float4 p, bool valid) {
            const bool nb = valid & (!SKIP || base + k != skip) & (dist2_exact(xi, p) < h2);
            mask |= (nb ? 1u : 0u) << k;
        };
        uint32_t k = 0;
        for (; k + 4 <= n; k += 4) {
            const float4 p0 = q(k), p1 = q(k + 1), p2 = q(k + 2), p3 = q(k + 3);
            test(k, p0, true);
            test(k + 1, p1, true);
            test(k + 2, p2, true);
            test(k + 3, p3, true);
        }
        if (k < n) {   // one to three left: load them together (repeats of the last one stay in range)
            const uint32_t r = n - k;
            const float4 p0 = q(k), p1 = q(k + (r > 1u ? 1 : 0)), p2 = q(k + (r > 2u ? 2 : 0));
            test(k, p0, true);
            test(k + 1, p1, r > 1u);
            test(k + 2, p2, r > 2u);
        }
        append_mask(mask, base, chunk, nf, cap, cnt, buf);
    }
}

// Neighbour passes run L (1, 2, 4 or 8) lanes per particle: lane q of the group
// takes list entries k = q, q+L, q+2L, ...  The lanes of a wave instruction
// that belong to one particle read adjacent entries of one 16-byte chunk of
// its list, and a gather instruction touches the neighbours of 64/L
// particles, which share far fewer cache lines than those of 64 (the address
// unit, not HBM, bounds the gather-heavy passes).  Per-lane partial sums are
// combined by group_sum in a fixed order.
template <int L>
__device__ __forceinline__ float group_sum(float v) {
    if (L >= 2) v += __shfl_xor(v, 1, 64);
    if (L >= 4) v += __shfl_xor(v, 2, 64);
    if (L >= 8) v += __shfl_xor(v, 4, 64);
    return v;
}

// lane position in its particle's group, and the particle
template <int L>
__device__ __forceinline__ int64_t group_particle(int& q) {
    const int64_t g = particle_index();
    q = (int)(g & (L - 1));
    return g / L;
}

template <int L, class F>
__device__ __forceinline__ void for_each_nbr_l(const uint32_t* __restrict__ list, int64_t nf, int64_t i, int q,
                                               uint32_t n, F&& f) {
    static_assert(L == 1 || L == 2 || L == 4 || L == 8, "lanes per particle");
    if (L == 1) {
        for_each_nbr(list, nf, i, n, f);
        return;
    }
    // entry k of particle i sits at list + 4 ((k/4) nf + i) + k%4; this lane
    // takes k = q + L t.  Four of its entries per round, loaded ahead of the
    // work: for L = 2 two chunks hold them (positions q and q + 2), for
    // L >= 4 one chunk row each, L/4 rows apart.
    const int64_t step = nf << 2;   // one chunk row
    const uint32_t* p = list + ((((int64_t)(q >> 2) * nf + i) << 2) + (q & 3));
    const uint4* p4 = reinterpret_cast<const uint4*>(list) + i;   // L = 2: whole chunks
    uint32_t k = (uint32_t)q;
    for (; k + 3 * L < n; k += 4 * L) {
        uint32_t j[4];
        if (L == 2) {   // both lanes load the two chunks (one load each instead of two) and pick their entries
            const uint4 a = p4[0], b = p4[nf];
            j[0] = q ? a.y : a.x;
            j[1] = q ? a.w : a.z;
            j[2] = q ? b.y : b.x;
            j[3] = q ? b.w : b.z;
            p4 += 2 * nf;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) j[u] = p[u * (L / 4) * step];
            p += 4 * (L / 4) * step;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) f(j[u]);
    }
    if (L == 2) {   // up to three left, k, k+2 (this chunk row) and k+4 (the next)
        if (k < n) {
            const uint4 a = p4[0];
            f(q ? a.y : a.x);
            if (k + 2 < n) f(q ? a.w : a.z);
            if (k + 4 < n) {
                const uint4 b = p4[nf];
                f(q ? b.y : b.x);
            }
        }
        return;
    }
    for (; k < n; k += L) f(list[(((int64_t)(k >> 2) * nf + i) << 2) + (k & 3u)]);
}

// scan_with on candidates read from global memory
template <bool SKIP>
__device__ __forceinline__ void scan_candidates(const float4* __restrict__ pos, uint32_t b, uint32_t e, float4 xi,
                                                uint32_t skip, float h2, uint4*& chunk, int64_t nf, int32_t cap,
                                                uint32_t& cnt, uint4& buf) {
    scan_with<SKIP>([&](uint32_t c) { return pos[c]; }, b, e, xi, skip, h2, chunk, nf, cap, cnt, buf);
}

// A wave's window of candidates staged in LDS: entry t of the window sits at
// slot t + t/8 (one pad slot per eight spreads the lanes' reads of
// neighbouring cells over the banks).
constexpr uint32_t kWinCand = 192;
constexpr uint32_t kWinSlots = kWinCand + kWinCand / 8 + 4;   // + a group's overhang past the last entry
__device__ __forceinline__ uint32_t win_slot(uint32_t t) { return t + (t >> 3); }

// scan_with over the candidates [b, e) of a window staged from wb on: the
// groups of four start at multiples of four in the window, so a group's
// slots are contiguous (its four entries never straddle a pad) and load at
// fixed offsets from one address.  The group holding b may start before it
// and the last may run past e (at most three slots past the window's last
// entry, inside kWinSlots): those candidates are loaded but never accepted.
template <bool SKIP>
__device__ __forceinline__ void scan_window(const float4* __restrict__ win, uint32_t wb, uint32_t b, uint32_t e,
                                            float4 xi, uint32_t skip, float h2, uint4*& chunk, int64_t nf,
                                            int32_t cap, uint32_t& cnt, uint4& buf) {
    if (b >= e) return;
    for (uint32_t base = wb + ((b - wb) & ~3u); base < e; base += 32u) {
        const uint32_t n = min(e - base, 32u);
        uint32_t mask = 0u;
        for (uint32_t k = 0; k < n; k += 4) {
            const float4* g = win + win_slot(base - wb + k);
            const float4 p[4] = {g[0], g[1], g[2], g[3]};
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) mask |= (dist2_exact(xi, p[j]) < h2 ? 1u : 0u) << (k + j);
        }
        // keep the bits of [b, e), without the particle itself
        const uint32_t lo = b > base ? b - base : 0u, hi = e - base;
        uint32_t keep = (hi >= 32u ? ~0u : (1u << hi) - 1u) & ~((1u << lo) - 1u);
        if (SKIP && skip - base < 32u) keep &= ~(1u << (skip - base));
        append_mask(mask & keep, base, chunk, nf, cap, cnt, buf);
    }
}

// LDS written by some lanes of a wave and read by others: order the two
// (the LDS executes one wave's instructions in order; this keeps the
// compiler from moving them across each other)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Store the partial last chunk of a list filled by scan_candidates: its k
// entries sit in the last k slots of buf.
__device__ __forceinline__ void list_flush(uint4* chunk, int32_t cap, uint32_t cnt, uint4 buf) {
    const uint32_t k = min(cnt, (uint32_t)cap) & 3u;
    if (k == 0u) return;
    uint4 o = buf;
    if (k == 1u) o = make_uint4(buf.w, 0u, 0u, 0u);
    if (k == 2u) o = make_uint4(buf.z, buf.w, 0u, 0u);
    if (k == 3u) o = make_uint4(buf.y, buf.z, buf.w, 0u);
    *chunk = o;
}

}  // namespace
}  // namespace sph
