// HIP kernels of the TLSPH damage step for gfx950 (MI355X).
//
// Data layout (all per-particle arrays in Hilbert order of their cells,
// stride np, a multiple of 64): field component c of particle i at
// [c * np + i].  The neighbour list is "sliced": the 64 particles of slice
// s = i / 64 keep their k-th neighbour at col[slice_ptr[s] + 64 k + (i % 64)],
// so the 64 lanes of a wavefront read 64 consecutive indices per neighbour
// step.  One lane owns one particle and sums its neighbours in a fixed order:
// no floating-point atomics anywhere, results independent of the launch
// shape.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "tlsph_internal.h"
#include "tlsph_math.h"

namespace tlsph {

// ===========================================================================
// neighbour-list build (Sec. 2: S_i fixed in the reference configuration)
// ===========================================================================

// Position of cell (x, y, z) along a three-dimensional Hilbert curve over
// 2^kCellBits cells per axis: the coordinates are turned into the curve's
// index in transposed form (Skilling's method: undo the excess rotations and
// reflections from the top bit down, then Gray-decode), whose bits are then
// interleaved, highest level first.  Consecutive keys are face-adjacent
// cells, so a run of keys (a tile) is a compact region; a run of Morton keys
// may jump across the domain, which puts more of a tile's neighbours outside
// it.
__device__ __forceinline__ uint64_t cell_key(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t X[3] = {x, y, z};
    for (uint32_t Q = 1u << (kCellBits - 1); Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = 1u << (kCellBits - 1); Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    uint64_t key = 0;
    for (int b = kCellBits - 1; b >= 0; --b)
#pragma unroll
        for (int i = 0; i < 3; ++i) key = (key << 1) | (((X[i] ^ t) >> b) & 1u);
    return key;
}

// Per-specimen record of 8 doubles (caller order, particles contiguous per
// specimen): bounding box lo[3], hi[3], then 1 / cell edge.  The edge is the
// specimen's h, or with graded spacing the largest support h_per_spacing
// (max V0)^(1/3), each a hair larger so that pairs closer than the support
// never sit two cells apart after rounding.
constexpr int kBBox = 8;
__global__ void k_bbox(const double* __restrict__ X, const double* __restrict__ V0, int64_t n,
                       const int64_t* __restrict__ off, const DevSpec* __restrict__ specs,
                       double* __restrict__ bbox) {
    __shared__ double red[7][256];
    const int s = blockIdx.x;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, vmax = 0.0;
    for (int64_t i = off[s] + threadIdx.x; i < off[s + 1]; i += blockDim.x) {
        for (int c = 0; c < 3; ++c) {
            const double x = X[c * n + i];
            lo[c] = x < lo[c] ? x : lo[c];
            hi[c] = x > hi[c] ? x : hi[c];
        }
        vmax = V0[i] > vmax ? V0[i] : vmax;
    }
    for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = lo[c];
        red[3 + c][threadIdx.x] = hi[c];
    }
    red[6][threadIdx.x] = vmax;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int c = 0; c < 3; ++c) {
                red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + w]);
                red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + w]);
            }
            red[6][threadIdx.x] = fmax(red[6][threadIdx.x], red[6][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) bbox[kBBox * s + threadIdx.x] = red[threadIdx.x][0];
    if (threadIdx.x == 6) {
        const DevSpec& P = specs[s];
        bbox[kBBox * s + 6] = P.h_per_spacing > 0.0
                                  ? 1.0 / (P.h_per_spacing * cbrt(red[6][0]) * (1.0 + 1e-9))
                                  : P.inv_cell;
        bbox[kBBox * s + 7] = 0.0;
    }
}

__device__ __forceinline__ int spec_of(const int64_t* off, int n_spec, int64_t i) {
    int lo = 0, hi = n_spec;  // largest s with off[s] <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void cell_of(const double* bb, double x, double y, double z,
                                        int32_t c[3]) {
    const double xs[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        const double q = floor((xs[a] - bb[a]) * bb[6]);
        c[a] = q < 0.0 ? 0 : (int32_t)q;
    }
}

__global__ void k_keys(const double* __restrict__ X, int64_t n, int64_t n_pow2,
                       const int64_t* __restrict__ off, int n_spec,
                       const double* __restrict__ bbox, uint64_t* __restrict__ keys,
                       int32_t* __restrict__ vals, int32_t* __restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pow2) return;
    if (i >= n) {
        keys[i] = ~0ull;
        vals[i] = 0x7fffffff;
        return;
    }
    const int s = spec_of(off, n_spec, i);
    int32_t c[3];
    cell_of(bbox + kBBox * s, X[i], X[n + i], X[2 * n + i], c);
    if (c[0] >= (1 << kCellBits) || c[1] >= (1 << kCellBits) || c[2] >= (1 << kCellBits))
        atomicOr(&err[3], 1);
    keys[i] = ((uint64_t)s << kSpecShift) | cell_key(c[0], c[1], c[2]);
    vals[i] = (int32_t)i;
}

// one compare-exchange stage of a bitonic sort of (key, val) pairs
__global__ void k_bitonic(uint64_t* __restrict__ keys, int32_t* __restrict__ vals, int64_t N,
                          int64_t j, int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const uint64_t ka = keys[i], kb = keys[l];
    const int32_t va = vals[i], vb = vals[l];
    const bool a_gt_b = (ka > kb) || (ka == kb && va > vb);
    const bool asc = (i & k) == 0;
    if (a_gt_b == asc) {
        keys[i] = kb; keys[l] = ka;
        vals[i] = vb; vals[l] = va;
    }
}

// The stages of the same sort whose partners lie within one block of kSortB
// elements (j < kSortB), run in LDS: with k <= kSortB every stage of the
// network from k = 2 (the block's own sort), else the stages j < kSortB of
// the merge of size k.  Blocks of kSortB / 2 threads, one pair per stage each;
// N (a power of two) below kSortB makes one block of N elements.
constexpr int kSortB = 2048;
__global__ void __launch_bounds__(kSortB / 2) k_bitonic_lds(uint64_t* __restrict__ keys,
                                                            int32_t* __restrict__ vals, int64_t N,
                                                            int64_t k_merge) {
    __shared__ uint64_t sk[kSortB];
    __shared__ int32_t sv[kSortB];
    const int B = (int)(N < kSortB ? N : kSortB);
    const int64_t base = (int64_t)blockIdx.x * B;
    for (int e = threadIdx.x; e < B; e += blockDim.x) {
        sk[e] = keys[base + e];
        sv[e] = vals[base + e];
    }
    __syncthreads();
    const int64_t k_lo = k_merge > 0 ? k_merge : 2;
    const int64_t k_hi = k_merge > 0 ? k_merge : B;
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = (k >> 1 < B ? k >> 1 : B >> 1); j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < B / 2; t += blockDim.x) {
                // the t-th pair (e, e + j) of the stage
                const int e = (int)(((t / j) * 2 * j) + (t % j));
                const int l = e + (int)j;
                const uint64_t ka = sk[e], kb = sk[l];
                const int32_t va = sv[e], vb = sv[l];
                const bool a_gt_b = (ka > kb) || (ka == kb && va > vb);
                const bool asc = ((base + e) & k) == 0;
                if (a_gt_b == asc) {
                    sk[e] = kb; sk[l] = ka;
                    sv[e] = vb; sv[l] = va;
                }
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < B; e += blockDim.x) {
        keys[base + e] = sk[e];
        vals[base + e] = sv[e];
    }
}

// Sort N (a power of two, >= 2) (key, val) pairs ascending by key, then val:
// the bitonic network, its stages with partners closer than kSortB run in
// LDS, the others one launch each.
hipError_t launch_bitonic_sort(uint64_t* keys, int32_t* vals, int64_t N, hipStream_t st) {
    constexpr int T = 256;
    const int B = (int)(N < kSortB ? N : kSortB);
    const unsigned blocks = (unsigned)(N / B);
    k_bitonic_lds<<<blocks, B / 2, 0, st>>>(keys, vals, N, 0);
    for (int64_t k = 2 * (int64_t)B; k <= N; k <<= 1) {
        for (int64_t j = k >> 1; j >= B; j >>= 1)
            k_bitonic<<<(unsigned)((N + T - 1) / T), T, 0, st>>>(keys, vals, N, j, k);
        k_bitonic_lds<<<blocks, B / 2, 0, st>>>(keys, vals, N, k);
    }
    return hipGetLastError();
}

__global__ void k_apply_perm(DevState s, const double* __restrict__ X_in,
                             const double* __restrict__ V0_in, const int32_t* __restrict__ bc_in,
                             const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                             D4* __restrict__ XV, int32_t* __restrict__ specs_out,
                             int32_t* __restrict__ bcs, int32_t* __restrict__ perm,
                             int32_t* __restrict__ iperm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.np) return;
    const int64_t n = s.n;
    if (p < n) {
        const int32_t o = vals[p];
        perm[p] = o;
        iperm[o] = (int32_t)p;
        XV[p] = D4{X_in[o], X_in[n + o], X_in[2 * n + o], V0_in[o]};
        int32_t g = bc_in[o];
        if (g < -1 || g >= s.n_bc) {  // reported as an argument error by the host
            atomicOr(&s.err[3], 2);
            g = -1;
        }
        bcs[p] = g;
        const int32_t sp = (int32_t)(keys[p] >> kSpecShift);
        specs_out[p] = sp;
        const DevSpec& P = s.specs[sp];
        s.hs[p] = P.h_per_spacing > 0.0 ? P.h_per_spacing * cbrt(V0_in[o]) : P.h;
        s.arad[p] = 0.5 * cbrt(V0_in[o]);
    } else {
        perm[p] = -1;
        s.hs[p] = 0.0;
        s.arad[p] = 0.0;
        XV[p] = D4{0.0, 0.0, 0.0, 0.0};
        bcs[p] = -1;
        specs_out[p] = 0;
    }
}

// sorted particle range of every specimen
__global__ void k_spec_ranges(DevSpec* specs, int n_spec, const uint64_t* __restrict__ keys,
                              int64_t n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_spec) return;
    auto lower = [&](uint64_t key) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < key) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    specs[s].first = lower((uint64_t)s << kSpecShift);
    specs[s].last = lower((uint64_t)(s + 1) << kSpecShift);
}

// Visit the neighbours of sorted particle p over the 27 cells around it, in
// a fixed order.  The distance test is evaluated exactly as written (no
// fused multiply-add) so membership is decided identically to a plain
// evaluation of |X_j - X_i|^2 < h^2.
template <typename F>
__device__ __forceinline__ int for_neighbours(const DevState& s, const uint64_t* keys,
                                              const double* bbox, int64_t p, F&& visit) {
#pragma clang fp contract(off)
    const int sp = s.spec[p];
    const DevSpec& P = s.specs[sp];
    const D4 xp = s.XV[p];
    const double xi = xp.x, yi = xp.y, zi = xp.z;
    int32_t c[3];
    cell_of(bbox + kBBox * sp, xi, yi, zi, c);
    const double hp = s.hs[p];
    int count = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int32_t cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= (1 << kCellBits) ||
                    cy >= (1 << kCellBits) || cz >= (1 << kCellBits))
                    continue;
                const uint64_t key = ((uint64_t)sp << kSpecShift) | cell_key(cx, cy, cz);
                int64_t lo = P.first, hi = P.last;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (keys[mid] < key) lo = mid + 1; else hi = mid;
                }
                for (int64_t q = lo; q < P.last && keys[q] == key; ++q) {
                    if (q == p) continue;
                    const D4 xq = s.XV[q];
                    const double d0 = xq.x - xi;
                    const double d1 = xq.y - yi;
                    const double d2 = xq.z - zi;
                    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    double lim = P.h2;
                    if (s.var_h) {   // graded spacing: the pair's support (h_p + h_q) / 2
                        const double hpq = 0.5 * (hp + s.hs[q]);
                        lim = hpq * hpq;
                    }
                    if (r2 < lim) visit(count++, (int32_t)q);
                }
            }
    return count;
}

__global__ void k_count(DevState s, const uint64_t* __restrict__ keys,
                        const double* __restrict__ bbox, int32_t* __restrict__ nnb) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.np) return;
    if (p >= s.n) {
        nnb[p] = 0;
        return;
    }
    const int cnt = for_neighbours(s, keys, bbox, p, [](int, int32_t) {});
    nnb[p] = cnt;
    atomicMax(&s.err[1], cnt);
}

// slice_ptr[t] = sum over earlier slices of 64 * (max count in the slice);
// one block, fixed order.
__global__ void __launch_bounds__(1024) k_slice_scan(const int32_t* __restrict__ nnb,
                                                     int64_t n_slices,
                                                     int64_t* __restrict__ slice_ptr) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n_slices + 1023) / 1024;
    const int64_t a = t * per, b = (a + per < n_slices) ? a + per : n_slices;
    int64_t sum = 0;
    for (int64_t q = a; q < b; ++q) {
        int w = 0;
        for (int l = 0; l < kSlice; ++l) w = max(w, nnb[q * kSlice + l]);
        sum += (int64_t)w * kSlice;
    }
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int q = 0; q < 1024; ++q) {
            const int64_t v = part[q];
            part[q] = run;
            run += v;
        }
        slice_ptr[n_slices] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t q = a; q < b; ++q) {
        slice_ptr[q] = run;
        int w = 0;
        for (int l = 0; l < kSlice; ++l) w = max(w, nnb[q * kSlice + l]);
        run += (int64_t)w * kSlice;
    }
}

__global__ void k_fill(DevState s, const uint64_t* __restrict__ keys,
                       const double* __restrict__ bbox, int32_t* __restrict__ col,
                       int64_t cap_slots) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.np) return;
    if (s.slice_ptr[s.np / kSlice] > cap_slots) return;  // capacity error reported by the host
    const int64_t sl = p / kSlice;
    const int w = (int)((s.slice_ptr[sl + 1] - s.slice_ptr[sl]) / kSlice);
    int32_t* base = col + s.slice_ptr[sl] + (p % kSlice);
    int cnt = 0;
    if (p < s.n)
        cnt = for_neighbours(s, keys, bbox, p,
                             [&](int k, int32_t q) { base[(int64_t)k * kSlice] = q; });
    // the rest of the slice's width points at the particle itself (a valid
    // address for loops that run to the slice width and mask the excess)
    const int32_t self = p < s.n ? (int32_t)p : 0;
    for (int k = cnt; k < w; ++k) base[(int64_t)k * kSlice] = self;
}

// Correction matrix L_i = sum_j V_j (X_j - X_i) (x) gradW_ij (eq.
// correction_matrix) and its inverse, in double.
__global__ void k_shape(DevState s, double* __restrict__ Linv, float* __restrict__ Linv32) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.np) return;
    const int64_t np = s.np;
    if (p >= s.n) {
        for (int k = 0; k < 9; ++k) {
            Linv[k * np + p] = 0.0;
            if (Linv32) Linv32[k * np + p] = 0.0f;
        }
        return;
    }
    if (s.slice_ptr[np / kSlice] > s.col_cap) return;  // list did not fit: never read col
    const DevSpec& P = s.specs[s.spec[p]];
    const D4 xp = s.XV[p];
    double L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int cnt = s.nnb[p];
    const int32_t* cp = s.col + s.slice_ptr[p / kSlice] + (p % kSlice);
    for (int k = 0; k < cnt; ++k) {
        const int32_t j = cp[(int64_t)k * kSlice];
        const D4 xj = s.XV[j];
        const double d[3] = {xj.x - xp.x, xj.y - xp.y, xj.z - xp.z};
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double W, dW;
        if (s.var_h) {   // the pair's support
            const double h = 0.5 * (s.hs[p] + s.hs[j]);
            spline(r, 1.0 / h, 8.0 / (M_PI * h * h * h), W, dW);
        } else {
            spline(r, P.inv_h, P.wnorm, W, dW);
        }
        const double g = xj.w * dW / r;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) L[3 * a + b] += d[a] * g * d[b];
    }
    double nrm = 0.0;
    for (int k = 0; k < 9; ++k) nrm += L[k] * L[k];
    nrm = sqrt(nrm);
    const double det = det33(L);
    double Li[9];
    if (!(fabs(det) > 1e-12 * nrm * nrm * nrm)) {
        atomicMin(&s.err[0], (int32_t)p);
        for (int k = 0; k < 9; ++k) Li[k] = 0.0;
    } else {
        inv33(L, Li);
    }
    for (int k = 0; k < 9; ++k) {
        Linv[k * np + p] = Li[k];
        if (Linv32) Linv32[k * np + p] = (float)Li[k];
    }
}

// initial state: u = 0, v = 0, F = I, stresses and accumulators 0, f = f0,
// D = q1 f*(f0) under GTN, Q = 0, t = 0
__global__ void k_init(DevState s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < s.n_spec) s.t[p] = 0.0;
    if (p >= s.np) return;
    const int64_t np = s.np;
    const DevSpec& P = s.specs[s.spec[p]];
    const double D0 = (P.damage == 3) ? gtn_D(P, P.f0) : 0.0;
    s.U[0][p] = D4{0.0, 0.0, 0.0, 0.0};
    s.U[1][p] = D4{0.0, 0.0, 0.0, 0.0};
    s.VW[p] = D4{0.0, 0.0, 0.0, s.XV[p].w * (1.0 - D0)};
    for (int c = 0; c < 3; ++c) {
        s.force[c * np + p] = 0.0;
        s.fvisc[c * np + p] = 0.0;
    }
    s.ccnt[p] = 0;
    if (s.GQ) {
        GQRec<double> g;
        GHRec<double> h;
        for (int k = 0; k < 9; ++k) { g.q[k] = 0.0; h.h[k] = 0.0; }
        g.omd = 1.0 - D0;
        h.pad = 0.0;
        s.GQ[p] = g;
        s.GH[p] = h;
    } else {
        GQRec<float> g;
        GHRec<float> h;
        for (int k = 0; k < 9; ++k) { g.q[k] = 0.0f; h.h[k] = 0.0f; }
        g.omd = (float)(1.0 - D0);
        h.pad = 0.0f;
        s.GQ32[p] = g;
        s.GH32[p] = h;
    }
    for (int k = 0; k < 6; ++k) {
        if (s.sig) s.sig[k * np + p] = 0.0;
        if (s.sig32) s.sig32[k * np + p] = 0.0f;
    }
    s.eps_p[p] = 0.0;
    s.eps_rate[p] = 0.0;
    s.d_init[p] = 0.0;
    s.w_p[p] = 0.0;
    s.e[p] = 0.0;
    s.f_void[p] = P.f0;
    s.D[p] = D0;
}

hipError_t launch_build_count(DevState& s, const BuildBuffers& b, hipStream_t st) {
    const int T = 256;
    k_bbox<<<s.n_spec, 256, 0, st>>>(b.X_in, b.V0_in, s.n, b.spec_off, s.specs, b.bbox);
    k_keys<<<(unsigned)((b.n_pow2 + T - 1) / T), T, 0, st>>>(b.X_in, s.n, b.n_pow2, b.spec_off,
                                                             s.n_spec, b.bbox, b.keys, b.vals,
                                                             s.err);
    hipError_t e = launch_bitonic_sort(b.keys, b.vals, b.n_pow2, st);
    if (e != hipSuccess) return e;
    const unsigned gp = (unsigned)((s.np + T - 1) / T);
    k_apply_perm<<<gp, T, 0, st>>>(s, b.X_in, b.V0_in, b.bc_in, b.keys, b.vals,
                                   const_cast<D4*>(s.XV), const_cast<int32_t*>(s.spec),
                                   const_cast<int32_t*>(s.bc), const_cast<int32_t*>(s.perm),
                                   const_cast<int32_t*>(s.iperm));
    k_spec_ranges<<<(s.n_spec + 63) / 64, 64, 0, st>>>(const_cast<DevSpec*>(s.specs), s.n_spec,
                                                      b.keys, s.n);
    k_count<<<gp, T, 0, st>>>(s, b.keys, b.bbox, const_cast<int32_t*>(s.nnb));
    k_slice_scan<<<1, 1024, 0, st>>>(s.nnb, s.np / kSlice, const_cast<int64_t*>(s.slice_ptr));
    return hipGetLastError();
}

// One workgroup per tile of kTile particles: sort the tile's neighbour
// entries that lie outside the tile (bitonic, in LDS), keep each index once
// (the halo, ascending), then give every neighbour entry its local slot:
// j - start inside the tile, T + position in the halo outside.
__global__ void __launch_bounds__(256) k_halo(DevState s, int k_cap, int E,
                                              int32_t* __restrict__ halo,
                                              int32_t* __restrict__ halo_cnt,
                                              uint16_t* __restrict__ lcol) {
    extern __shared__ int32_t sh[];
    int32_t* srt = sh;            // [E]
    int32_t* hl = sh + E;         // [E]
    int32_t* part = sh + 2 * E;   // [257]
    const int tid = threadIdx.x;
    const int T = s.tile;                  // particles per tile (<= 256 threads)
    const int64_t t = blockIdx.x;
    const int64_t start = t * T;
    const int64_t end = start + T < s.n ? start + T : s.n;
    for (int e = tid; e < E; e += 256) srt[e] = 0x7fffffff;
    __syncthreads();
    const int64_t p = start + tid;
    const bool mine = tid < T;             // thread tid holds particle start + tid
    int cnt = 0;
    const int32_t* cp = nullptr;
    if (mine && p < s.n) {
        cnt = s.nnb[p];
        cp = s.col + s.slice_ptr[p / kSlice] + (p % kSlice);
        for (int k = 0; k < cnt; ++k) {
            const int32_t j = cp[(int64_t)k * kSlice];
            if (j < start || j >= end) srt[tid * k_cap + k] = j;
        }
    }
    __syncthreads();
    for (int k = 2; k <= E; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int e = tid; e < E; e += 256) {
                const int l = e ^ j;
                if (l > e) {
                    const int32_t a = srt[e], b = srt[l];
                    if ((a > b) == ((e & k) == 0)) {
                        srt[e] = b;
                        srt[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    const int per = E / 256;
    int c = 0;
    for (int e = tid * per; e < (tid + 1) * per; ++e) {
        const int32_t v = srt[e];
        if (v != 0x7fffffff && (e == 0 || srt[e - 1] != v)) ++c;
    }
    part[tid] = c;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int q = 0; q < 256; ++q) {
            const int v = part[q];
            part[q] = run;
            run += v;
        }
        part[256] = run;
    }
    __syncthreads();
    int pos = part[tid];
    for (int e = tid * per; e < (tid + 1) * per; ++e) {
        const int32_t v = srt[e];
        if (v != 0x7fffffff && (e == 0 || srt[e - 1] != v)) hl[pos++] = v;
    }
    __syncthreads();
    const int H = part[256];
    for (int h = tid; h < H; h += 256) halo[t * s.halo_cap + h] = hl[h];
    // past the count, n (no particle) for as far as a staging round reads
    const int pad_end = H + kHaloPad < s.halo_cap ? H + kHaloPad : s.halo_cap;
    for (int h = H + tid; h < pad_end; h += 256) halo[t * s.halo_cap + h] = (int32_t)s.n;
    if (tid == 0) {
        halo_cnt[t] = H;
        atomicMax(&s.err[4], H);
    }
    if (mine && p < s.np) {
        const int64_t sl = p / kSlice;
        const int w = (int)((s.slice_ptr[sl + 1] - s.slice_ptr[sl]) / kSlice);
        uint16_t* lp = lcol + s.slice_ptr[sl] + (p % kSlice);
        for (int k = cnt; k < w; ++k) lp[(int64_t)k * kSlice] = (uint16_t)tid;
    }
    if (mine && p < s.n) {
        uint16_t* lp = lcol + s.slice_ptr[p / kSlice] + (p % kSlice);
        for (int k = 0; k < cnt; ++k) {
            const int32_t j = cp[(int64_t)k * kSlice];
            int loc;
            if (j >= start && j < end) {
                loc = (int)(j - start);
            } else {
                int lo = 0, hi = H;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (hl[mid] < j) lo = mid + 1; else hi = mid;
                }
                loc = T + lo;
            }
            lp[(int64_t)k * kSlice] = (uint16_t)loc;
        }
    }
}

hipError_t launch_halo(const DevState& s, int k_cap, int T, int32_t* halo, int32_t* halo_cnt,
                       uint16_t* lcol, hipStream_t st) {
    if (T < 1 || T > kTile) return hipErrorInvalidValue;
    int E = 256;
    while (E < T * k_cap) E <<= 1;
    const size_t lds = (2 * (size_t)E + 257) * sizeof(int32_t);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_halo),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    DevState t = s;   // the kernel reads the tile size and list stride from it
    t.tile = T;
    t.halo_cap = T * k_cap;
    const unsigned tiles = (unsigned)((s.n + T - 1) / T);
    k_halo<<<tiles, 256, lds, st>>>(t, k_cap, E, halo, halo_cnt, lcol);
    return hipGetLastError();
}

// Only after the host has checked that the sliced list fits col.
hipError_t launch_build_fill(DevState& s, const BuildBuffers& b, hipStream_t st) {
    const int T = 256;
    const unsigned gp = (unsigned)((s.np + T - 1) / T);
    k_fill<<<gp, T, 0, st>>>(s, b.keys, b.bbox, const_cast<int32_t*>(s.col), s.col_cap);
    return hipGetLastError();
}

hipError_t launch_shape_and_init(const DevState& s, bool mixed, hipStream_t st) {
    const int T = 256;
    const unsigned gp = (unsigned)((s.np + T - 1) / T);
    k_shape<<<gp, T, 0, st>>>(s, const_cast<double*>(s.Linv),
                              mixed ? const_cast<float*>(s.Linv32) : nullptr);
    const int64_t m = s.np > s.n_spec ? s.np : s.n_spec;
    k_init<<<(unsigned)((m + T - 1) / T), T, 0, st>>>(s);
    return hipGetLastError();
}

// ===========================================================================
// the step
// ===========================================================================

// 1/sqrt(x): the hardware estimate refined by Newton-Raphson steps
// y <- y + y (1 - x y^2) / 2, two for double and one for float (each step
// doubles the number of correct bits).  Not correctly rounded: a few ulp.
// An estimate of 0 or infinity (x infinite or 0) is returned as it is.
__device__ __forceinline__ double rsqrt_nr(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    double y = y0;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return (y0 == 0.0 || __builtin_isinf(y0)) ? y0 : y;
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    const float y0 = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-x * y0, y0, 1.0f);
    const float y = fmaf(0.5f * y0, e, y0);
    return (y0 == 0.0f || __builtin_isinf(y0)) ? y0 : y;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Give XCD x a contiguous run of tiles instead, so the neighbour halos
// of adjacent tiles are shared through one L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nblk) {
    constexpr int64_t kXcd = 8;
    const int64_t q = nblk / kXcd, r = nblk % kXcd;
    const int64_t x = b % kXcd, k = b / kXcd;
    return x * q + (x < r ? x : r) + k;
}

// Tile `part` (of G per workgroup) of a staged pass's workgroup, -1 if none.
// Workgroups take groups of G consecutive tiles (XCD-contiguous: the groups
// an XCD runs are one range).  Under run control the grid still spans every
// tile, and the first workgroups take the listed tiles of running specimens,
// G at a time with the same mapping over the list; the others get -1 and
// return at once.
// (list: the pass's run-control list, null when off; count: its length)
__device__ __forceinline__ int64_t work_tile(const int32_t* list, const int32_t* count, int G,
                                             int part, int64_t n_tiles) {
    if (list) {
        const int64_t nw = *count;
        const int64_t ng = (nw + G - 1) / G;
        if ((int64_t)blockIdx.x >= ng) return -1;
        const int64_t k = xcd_tile(blockIdx.x, ng) * G + part;
        if (k >= nw) return -1;
        const int64_t t = list[k];
        return t < n_tiles ? t : -1;   // (a list of this tile size has none beyond)
    }
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x) * G + part;
    return t < n_tiles ? t : -1;
}

// A specimen that run control has stopped keeps its state.
__device__ __forceinline__ bool frozen(const DevState& s, int sp) {
    return s.done != nullptr && s.done[sp] != kRunning;
}
// The same test in two parts, so that a kernel can load the flag early and
// wait for it only where it decides: the word is loaded whether run control
// is on or not (then from the specimen index array, a valid address: a
// specimen sp < n has a particle sp).
__device__ __forceinline__ int32_t run_word(const DevState& s, int sp) {
    return (s.done != nullptr ? s.done : s.spec)[sp];
}
__device__ __forceinline__ bool frozen_word(const DevState& s, int32_t w) {
    return s.done != nullptr && w != kRunning;
}

template <typename R>
__device__ __forceinline__ GQRec<R>* gq_of(const DevState& s);
template <>
__device__ __forceinline__ GQRec<double>* gq_of<double>(const DevState& s) { return s.GQ; }
template <>
__device__ __forceinline__ GQRec<float>* gq_of<float>(const DevState& s) { return s.GQ32; }
template <typename R>
__device__ __forceinline__ GHRec<R>* gh_of(const DevState& s);
template <>
__device__ __forceinline__ GHRec<double>* gh_of<double>(const DevState& s) { return s.GH; }
template <>
__device__ __forceinline__ GHRec<float>* gh_of<float>(const DevState& s) { return s.GH32; }

// Everything the force pass needs of a neighbour (and of the particle
// itself): reference position and volume, displacement, 1 - D, Q = P L^-T
// and H = F - I.  Also the LDS record of the staged kernel.
template <typename R>
struct LRecB;
template <>
struct alignas(16) LRecB<double> {
    double x, y, z, V0, ux, uy, uz, omd;
    double q[9], h[9];
    double hs;   // support radius (graded spacing only; not in the LDS image)
};
template <>
struct alignas(16) LRecB<float> {
    double x, y, z, ux, uy, uz;   // positions and displacements stay double
    float V0, omd;
    float q[9], h[9];
    double hs;   // support radius (graded spacing only; not in the LDS image)
};

template <typename R>
__device__ __forceinline__ LRecB<R> make_recb(const D4& xv, const GQRec<R>& g, const GHRec<R>& h,
                                               const D4& u) {
    LRecB<R> r;
    r.x = xv.x; r.y = xv.y; r.z = xv.z; r.V0 = R(xv.w);
    r.ux = u.x; r.uy = u.y; r.uz = u.z; r.omd = g.omd;
#pragma unroll
    for (int k = 0; k < 9; ++k) { r.q[k] = g.q[k]; r.h[k] = h.h[k]; }
    return r;
}

template <typename R>
struct ForceAcc {
    R a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0, g0 = 0, g1 = 0, g2 = 0;
};

// 1/sqrt(x) and 1/x for x > 0 finite (the refinement of rsqrt_nr and rcp_nr
// without their 0/infinity passthrough: callers select the zero cases).
__device__ __forceinline__ double rsqrt_pos(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
}
__device__ __forceinline__ float rsqrt_pos(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
}
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float rcp_pos(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// One pair of the force pass, with the kernel's constant factors left out
// (w = W / c and s = h dW/dr / c with c = 8 / (pi h^3); the finish applies
// c / h to a and b and c to the hourglass sum):
//   a += V_j (1 - D_j) s X_ij / r,  b += V_j Q_j s X_ij / r,
//   g += (1 - D_j) V_j w (e_ij . x_ij) / (|X_ij|^2 |x_ij|^2) x_ij
// with e_ij . x_ij = ((H_i + H_j) X_ij) . x_ij / 2 - (u_j - u_i) . x_ij
// (the error vector (F_i + F_j) X_ij / 2 - x_ij with F = I + H).  A pair
// whose current separation is zero adds no hourglass force.  With graded
// spacing (kVarH) each pair has its own support h_ij = (h_i + h_j) / 2, so
// the constant factors c / h_ij and c = 8 / (pi h_ij^3) enter per pair and the
// finish applies none.
template <typename R, bool kVarH = false>
__device__ __forceinline__ void force_pair(const LRecB<R>& ni, const LRecB<R>& nj, R inv_h,
                                           ForceAcc<R>& A, bool live = true) {
    // a padding slot (live = false) gets 1/r = 1/|x|^2 = 0: every term it
    // adds is an exact zero
    const R dx = R(nj.x - ni.x), dy = R(nj.y - ni.y), dz = R(nj.z - ni.z);
    const R r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const R ir = live ? rsqrt_pos(r2) : R(0);
    R kg = R(1), kw = R(1);
    if constexpr (kVarH) {
        inv_h = rcp_nr(R(0.5 * (ni.hs + nj.hs)));
        kw = R(8.0 / M_PI) * inv_h * inv_h * inv_h;
        kg = kw * inv_h;
    }
    const R q = r2 * ir * inv_h;
    // cubic spline: with a = 1 - q and b = max(1/2 - q, 0), W / c = 2 a^3 -
    // 8 b^3 and h dW/dr / c = -6 a^2 + 24 b^2 (b = 0 beyond q = 1/2, where
    // seven pairs in eight lie).  FP64 evaluates it without a branch; the
    // mixed form keeps the two-branch form, which fits its register budget
    // of four waves per SIMD without spilling.
    R w, sl;
    if constexpr (sizeof(R) == 8) {
        const R a = R(1) - q;
        const R b = fmax(R(0.5) - q, R(0));
        const R a2 = a * a, b2 = b * b;
        sl = fma(R(24), b2, R(-6) * a2);
        w = fma(R(-8) * b2, b, (a + a) * a2);
    } else if (q < R(0.5)) {
        w = fma(q * q, fma(R(6), q, R(-6)), R(1));
        sl = q * fma(R(18), q, R(-12));
    } else {
        const R a = R(1) - q;
        const R a2 = a * a;
        w = (a + a) * a2;
        sl = R(-6) * a2;
    }
    const R Vj = nj.V0;
    R gv = sl * ir * Vj;
    if constexpr (kVarH) {
        gv *= kg;
        w *= kw;
    }
    const R gx = gv * dx, gy = gv * dy, gz = gv * dz;
    A.a0 = fma(nj.omd, gx, A.a0); A.a1 = fma(nj.omd, gy, A.a1); A.a2 = fma(nj.omd, gz, A.a2);
    A.b0 = fma(nj.q[0], gx, fma(nj.q[1], gy, fma(nj.q[2], gz, A.b0)));
    A.b1 = fma(nj.q[3], gx, fma(nj.q[4], gy, fma(nj.q[5], gz, A.b1)));
    A.b2 = fma(nj.q[6], gx, fma(nj.q[7], gy, fma(nj.q[8], gz, A.b2)));
    const R du0 = R(nj.ux - ni.ux), du1 = R(nj.uy - ni.uy), du2 = R(nj.uz - ni.uz);
    const R x0 = dx + du0, x1 = dy + du1, x2 = dz + du2;
    const R rc2 = fma(x0, x0, fma(x1, x1, x2 * x2));
    const R irc2 = (live && rc2 > R(0)) ? rcp_pos(rc2) : R(0);
    const R v0 = fma(ni.h[0] + nj.h[0], dx, fma(ni.h[1] + nj.h[1], dy, (ni.h[2] + nj.h[2]) * dz));
    const R v1 = fma(ni.h[3] + nj.h[3], dx, fma(ni.h[4] + nj.h[4], dy, (ni.h[5] + nj.h[5]) * dz));
    const R v2 = fma(ni.h[6] + nj.h[6], dx, fma(ni.h[7] + nj.h[7], dy, (ni.h[8] + nj.h[8]) * dz));
    const R hx = fma(v0, x0, fma(v1, x1, v2 * x2));
    const R ux = fma(du0, x0, fma(du1, x1, du2 * x2));
    const R ex = fma(R(0.5), hx, -ux);
    const R c = Vj * nj.omd * w * ex * (ir * ir) * irc2;
    A.g0 = fma(c, x0, A.g0); A.g1 = fma(c, x1, A.g1); A.g2 = fma(c, x2, A.g2);
}

template <typename R>
__device__ __forceinline__ ForceAcc<R> acc_sum(const ForceAcc<R>& x, const ForceAcc<R>& y) {
    ForceAcc<R> r;
    r.a0 = x.a0 + y.a0; r.a1 = x.a1 + y.a1; r.a2 = x.a2 + y.a2;
    r.b0 = x.b0 + y.b0; r.b1 = x.b1 + y.b1; r.b2 = x.b2 + y.b2;
    r.g0 = x.g0 + y.g0; r.g1 = x.g1 + y.g1; r.g2 = x.g2 + y.g2;
    return r;
}

// The value of lane l ^ m (m = 1 or 2) within each group of four lanes, by a
// DPP quad permutation (a VALU operand modifier: no LDS traffic).
template <int M>
__device__ __forceinline__ float quad_xor(float v) {
    static_assert(M == 1 || M == 2, "quad permutations for xor 1 and 2");
    constexpr int ctrl = M == 1 ? 0xB1 : 0x4E;   // quad_perm [1,0,3,2] / [2,3,0,1]
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false));
}
template <int M>
__device__ __forceinline__ double quad_xor(double v) {
    static_assert(M == 1 || M == 2, "quad permutations for xor 1 and 2");
    constexpr int ctrl = M == 1 ? 0xB1 : 0x4E;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int M, typename R>
__device__ __forceinline__ ForceAcc<R> acc_xor(const ForceAcc<R>& x) {
    ForceAcc<R> r;
    r.a0 = quad_xor<M>(x.a0); r.a1 = quad_xor<M>(x.a1); r.a2 = quad_xor<M>(x.a2);
    r.b0 = quad_xor<M>(x.b0); r.b1 = quad_xor<M>(x.b1); r.b2 = quad_xor<M>(x.b2);
    r.g0 = quad_xor<M>(x.g0); r.g1 = quad_xor<M>(x.g1); r.g2 = quad_xor<M>(x.g2);
    return r;
}

// Pair sums of one particle in the canonical order of the force pass:
// neighbour k feeds partial sum k mod kSub (each partial in increasing k) and
// the partials combine as (p0 + p1) + (p2 + p3).  S adjacent lanes share a
// particle (S = 1, 2 or 4), lane `sub` holding partials sub, sub + S, ...;
// every S rounds identically.  All lanes of the wave must call this (the
// partials are exchanged across lanes); lanes without a particle pass cnt = 0.
// The neighbour indices of a lane's first G groups (neighbours sub, sub + S,
// ... below G kSub), loaded apart so that a kernel can issue them before its
// staging: the pair loop then runs those groups without waiting on memory.
// Local slots (below 2^16, kPack) go two to a register.
template <int S, int G, bool kPack = false>
struct FirstIdx {
    static constexpr int NP = kSub / S;
    static constexpr int E = G * NP;   // entries, group-major
    uint32_t w[kPack ? (E + 1) / 2 : E];
    __device__ int at(int g, int t) const {
        const int e = g * NP + t;
        if constexpr (kPack)
            return (int)((e & 1) ? w[e >> 1] >> 16 : w[e >> 1] & 0xffffu);
        else
            return (int)w[e];
    }
};
template <int S, int G, bool kPack = false, typename IdxOf>
__device__ __forceinline__ FirstIdx<S, G, kPack> first_indices(int cnt, int sub, IdxOf idx) {
    using FI = FirstIdx<S, G, kPack>;
    FI f;
    const auto at = [&](int e) {
        const int k = (e / FI::NP) * kSub + sub + S * (e % FI::NP);
        return (uint32_t)idx(k < cnt ? k : 0);
    };
#pragma unroll
    for (int e = 0; e < FI::E; e += kPack ? 2 : 1) {
        if constexpr (kPack)
            f.w[e >> 1] = at(e) | (e + 1 < FI::E ? at(e + 1) << 16 : 0u);
        else
            f.w[e] = at(e);
    }
    return f;
}

template <typename R, int S, bool kVarH = false, int G, bool kPack, typename IdxOf, typename RecOf>
__device__ __forceinline__ ForceAcc<R> pair_sums(const LRecB<R>& ni, int cnt, int sub, R inv_h,
                                                 IdxOf idx, RecOf rec,
                                                 const FirstIdx<S, G, kPack>& first) {
    static_assert(kSub == 4 && (S == 1 || S == 2 || S == 4), "canonical order has 4 partials");
    static_assert(G >= 1, "at least the first group is preloaded");
    constexpr int NP = kSub / S;
    ForceAcc<R> A[NP];
    // the group after the preloaded ones goes out first: its latency is spent
    // behind them (longer lists then run their indices one group of kSub
    // ahead of the arithmetic)
    int q[NP];
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        const int k = G * kSub + sub + S * t;
        q[t] = idx(k < cnt ? k : 0);
    }
    // the preloaded groups, unrolled (a lane past its count is masked off)
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int k0 = g * kSub;
        if (k0 < cnt) {
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                const int k = k0 + sub + S * t;
                force_pair<R, kVarH>(ni, rec(first.at(g, t)), inv_h, A[t], k < cnt);
            }
        }
    }
    for (int k0 = G * kSub; k0 < cnt; k0 += kSub) {
        int cur[NP];
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            cur[t] = q[t];
            const int kn = k0 + kSub + sub + S * t;
            q[t] = idx(kn < cnt ? kn : 0);
        }
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            const int k = k0 + sub + S * t;
            force_pair<R, kVarH>(ni, rec(cur[t]), inv_h, A[t], k < cnt);
        }
    }
    if constexpr (S == 1) {
        return acc_sum(acc_sum(A[0], A[1]), acc_sum(A[2], A[3]));
    } else if constexpr (S == 2) {
        const ForceAcc<R> x = acc_sum(A[0], acc_xor<1>(A[0]));   // p0 + p1
        const ForceAcc<R> y = acc_sum(A[1], acc_xor<1>(A[1]));   // p2 + p3
        return acc_sum(x, y);
    } else {
        const ForceAcc<R> x = acc_sum(A[0], acc_xor<1>(A[0]));   // p0 + p1 | p2 + p3
        return acc_sum(x, acc_xor<2>(x));
    }
}

// Penalty contact force on particle i at its position (xi, yi, zi) at t^n:
// the Hertz law of two spheres of radii a_i, a_j over every listed candidate
// closer than a_i + a_j, except reference neighbours of the same specimen
// that are both intact; F = k (4/3) E* sqrt(a_i a_j / (a_i + a_j)) delta^(3/2)
// along x_ij, k the mean of the two factors, 1/E* the sum of the shares.
// Also flags a particle that has left the list's skin.
__device__ __forceinline__ void contact_force(const DevState& s, int64_t i, int par, int sp,
                                              double xi, double yi, double zi, double Di,
                                              double f[3]) {
    const int64_t np = s.np;
    f[0] = f[1] = f[2] = 0.0;
    const DevSpec& Pi = s.specs[sp];
    const double ai = s.arad[i];
    const D4* __restrict__ Uc = s.U[par];
    const D4 ui = Uc[i];
    const double b0 = ui.x - s.ubuild[i], b1 = ui.y - s.ubuild[np + i],
                 b2 = ui.z - s.ubuild[2 * np + i];
    if (4.0 * (b0 * b0 + b1 * b1 + b2 * b2) > s.contact_skin * s.contact_skin)
        atomicOr(&s.err[2], kErrContact);
    const int cnt = s.ccnt[i];
    for (int k = 0; k < cnt; ++k) {
        const uint32_t e = (uint32_t)s.ccol[(int64_t)k * np + i];
        const int32_t q = (int32_t)(e & 0x7fffffffu);
        const bool ref = (e >> 31) != 0;
        if (ref && Di < 1.0 && s.D[q] < 1.0) continue;
        const DevSpec& Pq = s.specs[s.spec[q]];
        const double kc = 0.5 * (Pi.contact_k + Pq.contact_k);
        if (!(kc > 0.0)) continue;
        const D4 xq = s.XV[q], uq = Uc[q];
        const double d0 = (xq.x + uq.x) - xi, d1 = (xq.y + uq.y) - yi, d2 = (xq.z + uq.z) - zi;
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const double aq = s.arad[q], rc = ai + aq;
        if (!(r2 < rc * rc) || !(r2 > 0.0)) continue;
        const double r = sqrt(r2), delta = rc - r;
        const double es = 1.0 / (Pi.contact_comp + Pq.contact_comp);
        const double F = kc * (4.0 / 3.0) * es * sqrt(ai * aq / rc) * delta * sqrt(delta);
        const double g = F / r;
        f[0] -= g * d0;
        f[1] -= g * d1;
        f[2] -= g * d2;
    }
}

// What the finish needs of a particle besides its record, loaded before the
// pair sums so that their latency is spent behind them.
struct FinishIn {
    double D, V, vx, vy, vz;
    double grad_k, hg_k, dt, dt_rho0;
    int32_t bc, wall;
};
template <bool kVarH = false>
__device__ __forceinline__ FinishIn finish_in(const DevState& s, int64_t i, const DevSpec& P) {
    const D4 v = s.VW[i];
    // graded spacing: the pair sums carry the kernel's constant factors
    return FinishIn{s.D[i], s.XV[i].w, v.x, v.y, v.z, kVarH ? 1.0 : P.grad_k,
                    kVarH ? -P.hg_alpha * P.E : P.hg_k, P.dt, P.dt_rho0, s.bc[i], P.has_wall};
}

// Nodal force, kick, prescribed velocities, failed particles at rest, drift,
// rigid wall; stores v, V0 (1 - D), u^{n+1} and (for groups) the force.  The
// force per unit volume f / V_i is formed first: the kick is dt / rho0 times
// it (m = rho0 V_i).
template <typename R>
__device__ __forceinline__ void force_finish(const DevState& s, int64_t i, int par, const DevSpec& P,
                                             int sp, const LRecB<R>& ni, const ForceAcc<R>& A,
                                             const FinishIn& fin) {
    const int64_t np = s.np;
    const double Di = fin.D;
    const R omDi = R(1.0 - Di);
    const R ck = R(fin.grad_k);
    const R hgk = R(fin.hg_k) * omDi;
    const double Vi = fin.V;
    double fv0 = double(ck * (ni.q[0] * A.a0 + ni.q[1] * A.a1 + ni.q[2] * A.a2 + omDi * A.b0) + hgk * A.g0);
    double fv1 = double(ck * (ni.q[3] * A.a0 + ni.q[4] * A.a1 + ni.q[5] * A.a2 + omDi * A.b1) + hgk * A.g1);
    double fv2 = double(ck * (ni.q[6] * A.a0 + ni.q[7] * A.a1 + ni.q[8] * A.a2 + omDi * A.b2) + hgk * A.g2);
    if (s.av) {   // the artificial viscous force of the last deformation pass
        const double iv = rcp_nr(Vi);
        fv0 += s.fvisc[i] * iv;
        fv1 += s.fvisc[np + i] * iv;
        fv2 += s.fvisc[2 * np + i] * iv;
    }
    if (s.contact) {   // penalty contact with the listed candidates
        double fc[3];
        contact_force(s, i, par, sp, ni.x + ni.ux, ni.y + ni.uy, ni.z + ni.uz, Di, fc);
        const double iv = rcp_nr(Vi);
        fv0 += fc[0] * iv;
        fv1 += fc[1] * iv;
        fv2 += fc[2] * iv;
    }
    const double dt = fin.dt;
    double v[3] = {fin.vx + fin.dt_rho0 * fv0, fin.vy + fin.dt_rho0 * fv1,
                   fin.vz + fin.dt_rho0 * fv2};
    const double xi = ni.x, yi = ni.y, zi = ni.z;
    const int g = fin.bc;
    if (g >= 0) {
        const DevBC& B = s.bcs[g];
        const double th = s.t[sp] + 0.5 * dt;
        const double ramp = B.tau > 0.0 ? 1.0 - exp(-th / B.tau) : 1.0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (B.mask & (1 << c))
                v[c] = B.v_max[c] * ramp + (B.grad[3 * c] * xi + B.grad[3 * c + 1] * yi +
                                            B.grad[3 * c + 2] * zi);
    }
    if (Di >= 1.0) v[0] = v[1] = v[2] = 0.0;
    double un[3] = {ni.ux + dt * v[0], ni.uy + dt * v[1], ni.uz + dt * v[2]};
    if (fin.wall) {
        const double xw[3] = {xi + un[0], yi + un[1], zi + un[2]};
        const double dn = xw[0] * P.wall_n[0] + xw[1] * P.wall_n[1] + xw[2] * P.wall_n[2] - P.wall_d;
        if (dn < 0.0) {
            un[0] = (xw[0] - dn * P.wall_n[0]) - xi;
            un[1] = (xw[1] - dn * P.wall_n[1]) - yi;
            un[2] = (xw[2] - dn * P.wall_n[2]) - zi;
            const double vn = v[0] * P.wall_n[0] + v[1] * P.wall_n[1] + v[2] * P.wall_n[2];
            if (vn < 0.0) {
                v[0] -= vn * P.wall_n[0];
                v[1] -= vn * P.wall_n[1];
                v[2] -= vn * P.wall_n[2];
            }
        }
    }
    s.VW[i] = D4{v[0], v[1], v[2], Vi * (1.0 - Di)};
    s.U[par ^ 1][i] = D4{un[0], un[1], un[2], 0.0};
    if ((s.flags & kFlagStoreForce) || g >= 0) {
        s.force[i] = Vi * fv0; s.force[np + i] = Vi * fv1; s.force[2 * np + i] = Vi * fv2;
    }
}

// Pass B (forces at t^n, kick, drift).  Nodal force of Sec. 3.1,
//   f_i = V_i sum_j V_j [(1 - D_j) Q_i + (1 - D_i) Q_j] gradW_ij,
// evaluated as V_i [Q_i a + (1 - D_i) b] with a = sum_j V_j (1 - D_j) gradW_ij
// and b = sum_j V_j Q_j gradW_ij, plus hourglass control: with the error
// vector e_ij = (F_i + F_j)/2 X_ij - x_ij and delta = e_ij . x_ij / |x_ij|,
//   f_i^HG = -alpha E (1 - D_i) V_i sum_j (1 - D_j) V_j W_ij delta / |X_ij|^2
//            x_ij / |x_ij|.
// Then v += dt f / m, prescribed velocities at t^{n+1/2}, D = 1 at rest,
// u^{n+1} = u^n + dt v (into the other displacement buffer), rigid wall, and
// the record (v, V0 (1 - D)) the deformation pass gathers.  This variant
// gathers neighbours straight from global memory.
template <typename R, int S, bool kVarH = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S < 2 ? S : 2, 8)))
k_pass_b(DevState s, int par) {
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / S;
    const int sub = (int)(t % S);
    const bool in = i < s.n;
    const int64_t ii = in ? i : 0;
    const int sp = s.spec[ii];
    const DevSpec& P = s.specs[sp];
    const D4* __restrict__ XV = s.XV;
    const D4* __restrict__ Uc = s.U[par];
    const GQRec<R>* __restrict__ GQ = gq_of<R>(s);
    const GHRec<R>* __restrict__ GH = gh_of<R>(s);
    LRecB<R> ni = make_recb<R>(XV[ii], GQ[ii], GH[ii], Uc[ii]);
    if constexpr (kVarH) ni.hs = s.hs[ii];
    const R inv_h = R(P.inv_h);
    const bool live = in && !frozen(s, sp);
    const int cnt = live ? s.nnb[i] : 0;
    const FinishIn fin = finish_in<kVarH>(s, ii, P);
    const int32_t* __restrict__ cp = s.col + s.slice_ptr[ii / kSlice] + (ii % kSlice);
    const auto idx = [&](int k) { return (int)cp[(int64_t)k * kSlice]; };
    const ForceAcc<R> A = pair_sums<R, S, kVarH>(
        ni, cnt, sub, inv_h, idx,
        [&](int j) {
            LRecB<R> r = make_recb<R>(XV[j], GQ[j], GH[j], Uc[j]);
            if constexpr (kVarH) r.hs = s.hs[j];
            return r;
        },
        first_indices<S, 1>(cnt, sub, idx));
    // the particle's own Q is needed only now: reread it (the compiler barrier
    // keeps the load here) rather than keep it in registers through the loop
    asm volatile("" ::: "memory");
    if (live && sub == 0)
        force_finish<R>(s, i, par, P, sp, make_recb<R>(XV[i], GQ[i], GH[i], Uc[i]), A, fin);
}

// Particle of slot m of a tile's LDS image: the tile's T particles from
// `start`, then its halo row hl (capacity cap), which holds n (no particle)
// for kHaloPad entries past the tile's halo count; n for slots past the
// image.  The row entry is loaded unconditionally, at an index inside the
// row, and blended in with masks, so that the staging's loads need neither
// the halo count nor a branch on a loaded value (which may be turned into a
// branch whose join waits for the load): the first round of a staging goes
// out before the count has arrived.
__device__ __forceinline__ int64_t slot_particle(int m, int T, int cap, int64_t start, int64_t n,
                                                 const int32_t* __restrict__ hl) {
    const int h = m - T;
    const int64_t hv = hl[h >= 0 && h < cap ? h : 0];
    const int64_t in_tile = -(int64_t)(h < 0), past = -(int64_t)(h >= cap);
    const int64_t g = ((start + m) & in_tile) | (hv & ~in_tile);
    return (n & past) | (g & ~past);
}

// Largest workgroup of the staged force pass with S lanes per particle: four
// lanes run tiles of at most 128 particles, so that the register budget
// stays at two waves per SIMD.
__host__ __device__ constexpr int staged_block_max(int S) { return S == 4 ? 512 : kTile * S; }

// LDS image of the force-pass records of one tile and its halo (M slots).
// FP64: one 208-byte record per slot (13 units of 16 bytes, an odd number, so
// the slots read by the lanes of one 128-bit access spread over the bank
// groups as consecutive slots do), every field at a fixed offset from the
// record's address.  Mixed: 128-byte records would put every slot's field at
// the same bank group, so the image is field-major there (unit f of slot m
// at f * M + m).
template <typename R>
struct LdsB;
template <>
struct LdsB<double> {
    static constexpr int kUnits = 13;   // 26 doubles
    __device__ static void put(double2* L, int, int m, const LRecB<double>& r) {
        double2* p = L + m * kUnits;
        p[0] = double2{r.x, r.y};
        p[1] = double2{r.z, r.V0};
        p[2] = double2{r.ux, r.uy};
        p[3] = double2{r.uz, r.omd};
        p[4] = double2{r.q[0], r.q[1]};
        p[5] = double2{r.q[2], r.q[3]};
        p[6] = double2{r.q[4], r.q[5]};
        p[7] = double2{r.q[6], r.q[7]};
        p[8] = double2{r.q[8], r.h[0]};
        p[9] = double2{r.h[1], r.h[2]};
        p[10] = double2{r.h[3], r.h[4]};
        p[11] = double2{r.h[5], r.h[6]};
        p[12] = double2{r.h[7], r.h[8]};
    }
    __device__ static LRecB<double> get(const double2* L, int, int m) {
        const double2* p = L + m * kUnits;
        LRecB<double> r;
        double2 t;
        t = p[0]; r.x = t.x; r.y = t.y;
        t = p[1]; r.z = t.x; r.V0 = t.y;
        t = p[2]; r.ux = t.x; r.uy = t.y;
        t = p[3]; r.uz = t.x; r.omd = t.y;
        t = p[4]; r.q[0] = t.x; r.q[1] = t.y;
        t = p[5]; r.q[2] = t.x; r.q[3] = t.y;
        t = p[6]; r.q[4] = t.x; r.q[5] = t.y;
        t = p[7]; r.q[6] = t.x; r.q[7] = t.y;
        t = p[8]; r.q[8] = t.x; r.h[0] = t.y;
        t = p[9]; r.h[1] = t.x; r.h[2] = t.y;
        t = p[10]; r.h[3] = t.x; r.h[4] = t.y;
        t = p[11]; r.h[5] = t.x; r.h[6] = t.y;
        t = p[12]; r.h[7] = t.x; r.h[8] = t.y;
        return r;
    }
};
template <>
struct LdsB<float> {
    static constexpr int kUnits = 8;    // 6 doubles + 20 floats
    __device__ static void put(double2* L, int M, int m, const LRecB<float>& r) {
        L[0 * M + m] = double2{r.x, r.y};
        L[1 * M + m] = double2{r.z, r.ux};
        L[2 * M + m] = double2{r.uy, r.uz};
        float4* F = reinterpret_cast<float4*>(L + 3 * M);
        F[0 * M + m] = float4{r.V0, r.omd, r.q[0], r.q[1]};
        F[1 * M + m] = float4{r.q[2], r.q[3], r.q[4], r.q[5]};
        F[2 * M + m] = float4{r.q[6], r.q[7], r.q[8], r.h[0]};
        F[3 * M + m] = float4{r.h[1], r.h[2], r.h[3], r.h[4]};
        F[4 * M + m] = float4{r.h[5], r.h[6], r.h[7], r.h[8]};
    }
    __device__ static LRecB<float> get(const double2* L, int M, int m) {
        LRecB<float> r;
        double2 t;
        t = L[0 * M + m]; r.x = t.x; r.y = t.y;
        t = L[1 * M + m]; r.z = t.x; r.ux = t.y;
        t = L[2 * M + m]; r.uy = t.x; r.uz = t.y;
        const float4* F = reinterpret_cast<const float4*>(L + 3 * M);
        float4 f;
        f = F[0 * M + m]; r.V0 = f.x; r.omd = f.y; r.q[0] = f.z; r.q[1] = f.w;
        f = F[1 * M + m]; r.q[2] = f.x; r.q[3] = f.y; r.q[4] = f.z; r.q[5] = f.w;
        f = F[2 * M + m]; r.q[6] = f.x; r.q[7] = f.y; r.q[8] = f.z; r.h[0] = f.w;
        f = F[3 * M + m]; r.h[1] = f.x; r.h[2] = f.y; r.h[3] = f.z; r.h[4] = f.w;
        f = F[4 * M + m]; r.h[5] = f.x; r.h[6] = f.y; r.h[7] = f.z; r.h[8] = f.w;
        return r;
    }
};

// The same pass with the tile's particles and its halo staged in LDS: the
// workgroup loads every record it needs once, then S lanes per particle run
// the pair sums from LDS through the 16-bit local neighbour slots.  Same
// arithmetic in the same order as the unstaged kernel, so results are bitwise
// identical.  Occupancy is bounded by LDS; S lanes per particle give the
// SIMDs several waves to switch between.
// Waves per SIMD the staged force pass must leave room for: two workgroups per
// CU need four (mixed form, two or four lanes per particle: tiles up to 196
// and 128 particles) or three (FP64, four lanes: tiles up to 96).  With graded
// spacing the mixed form needs more than 128 registers: three.
template <typename R, int S, bool kVarH = false>
__host__ __device__ constexpr int staged_waves_min() {
    return sizeof(R) == 4 && S >= 2 ? (kVarH ? 3 : 4) : (S == 4 ? 3 : 1);
}
// Whether the finish's inputs are loaded before the staging (their registers
// then live through the pair sums; the mixed form with two lanes has none to
// spare within its 128).
template <typename R, int S>
__host__ __device__ constexpr bool staged_finish_early() {
    return !(sizeof(R) == 4 && S == 2);
}

// Neighbour-index groups the staged force pass loads before its staging.
template <typename R, int S>
__host__ __device__ constexpr int staged_pre_groups() {
    return S == 1 ? 1 : sizeof(R) == 8 ? (S == 2 ? 6 : 2) : S == 2 ? 4 : 1;
}

// Graded spacing (kVarH): the slots' support radii follow the records in LDS
// (one double per slot).
template <typename R, int S, bool kVarH = false>
__global__ void __launch_bounds__(staged_block_max(S))
__attribute__((amdgpu_waves_per_eu(staged_waves_min<R, S, kVarH>(), 8))) k_pass_b_staged(DevState s, int par) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double2* __restrict__ L = reinterpret_cast<double2*>(lds_raw);
    const int M = s.lds_slots;
    double* __restrict__ Lhs = reinterpret_cast<double*>(L + (size_t)M * LdsB<R>::kUnits);
    const int T = s.tile;
    const int B = T * S;
    const int64_t tile = work_tile(s.tile_list, s.run_count, 1, 0, gridDim.x);
    if (tile < 0) return;
    const int64_t start = tile * T;
    const int32_t* __restrict__ hl = s.halo + tile * (int64_t)s.halo_cap;
    const D4* __restrict__ XV = s.XV;
    const D4* __restrict__ Uc = s.U[par];
    const GQRec<R>* __restrict__ GQ = gq_of<R>(s);
    const GHRec<R>* __restrict__ GH = gh_of<R>(s);
    // Two slots per thread per round, their index loads issued before their
    // record loads and those before the LDS stores.  The first round's halo
    // indices are loaded before anything else; the particle's own scalars, its
    // first neighbour slots and what its finish needs follow, so that their
    // latencies overlap those of the staging.  The first round needs no halo
    // count (slots past the image hold n): FP64 reads the count after it (two
    // memory latencies before the barrier); the mixed form reads it first.
    // Slots past the image, and past the particle count (last tile), load the
    // tile's first record and store nothing.
    const auto particle_of = [&](int m) { return slot_particle(m, T, s.halo_cap, start, s.n, hl); };
    int m0 = threadIdx.x;
    int64_t g0 = particle_of(m0), g1 = particle_of(m0 + B);
    const int pl = threadIdx.x / S;
    const int sub = threadIdx.x % S;
    const int64_t i = start + pl;
    const bool in = i < s.n;
    const int64_t ii = in ? i : start;
    // (the loads that others depend on first: count, slice start, specimen)
    const int cnt = in ? s.nnb[i] : 0;
    const int64_t slice0 = s.slice_ptr[ii / kSlice];
    const int sp = s.spec[ii];
    const DevSpec& P = s.specs[sp];
    const R inv_h = R(P.inv_h);
    const uint16_t* __restrict__ lp = s.lcol + slice0 + (ii % kSlice);
    const auto idx = [&](int k) { return (int)lp[(int64_t)k * kSlice]; };
    const auto first = first_indices<S, staged_pre_groups<R, S>(), true>(cnt, sub, idx);
    constexpr bool kEarly = staged_finish_early<R, S>();
    FinishIn fin_early;
    if constexpr (kEarly) fin_early = finish_in<kVarH>(s, ii, P);
    const auto stage = [&](int m0, int64_t g0, int64_t g1) {
        const int64_t l0 = g0 < s.n ? g0 : start, l1 = g1 < s.n ? g1 : start;
        const LRecB<R> r0 = make_recb<R>(XV[l0], GQ[l0], GH[l0], Uc[l0]);
        const LRecB<R> r1 = make_recb<R>(XV[l1], GQ[l1], GH[l1], Uc[l1]);
        double h0 = 0.0, h1 = 0.0;
        if constexpr (kVarH) {
            h0 = s.hs[l0];
            h1 = s.hs[l1];
        }
        if (g0 < s.n) {
            LdsB<R>::put(L, M, m0, r0);
            if constexpr (kVarH) Lhs[m0] = h0;
        }
        if (g1 < s.n) {
            LdsB<R>::put(L, M, m0 + B, r1);
            if constexpr (kVarH) Lhs[m0 + B] = h1;
        }
    };
    if constexpr (sizeof(R) == 8) {
        stage(m0, g0, g1);
        const int tot = T + s.halo_cnt[tile];
        for (m0 += 2 * B; m0 < tot; m0 += 2 * B) stage(m0, particle_of(m0), particle_of(m0 + B));
    } else {
        // (the mixed form: a plain loop, whose registers fit four waves per
        // SIMD with the preloaded slots)
        const int tot = T + s.halo_cnt[tile];
        for (; m0 < tot; m0 += 2 * B) {
            stage(m0, g0, g1);
            g0 = particle_of(m0 + 2 * B);
            g1 = particle_of(m0 + 3 * B);
        }
    }
    __syncthreads();
    const auto rec = [&](int m) {
        LRecB<R> r = LdsB<R>::get(L, M, m);
        if constexpr (kVarH) r.hs = Lhs[m];
        return r;
    };
    const LRecB<R> ni = rec(in ? pl : 0);
    const ForceAcc<R> A = pair_sums<R, S, kVarH>(ni, cnt, sub, inv_h, idx, rec, first);
    // the particle's own Q is needed only now: reread it rather than keep it
    // in registers through the pair loop (the image is not written after the
    // barrier above, so a compiler barrier suffices: waves go on to their
    // finish as their own sums end)
    asm volatile("" ::: "memory");
    if (in && sub == 0 && !frozen(s, sp))
        force_finish<R>(s, i, par, P, sp, LdsB<R>::get(L, M, pl), A,
                        kEarly ? fin_early : finish_in<kVarH>(s, i, P));
}

// Pass A (deformation and constitutive update to t^{n+1}).
//   dF/dt_i = sum_j V_j (1 - D_j)(v_j - v_i) (x) gradW_ij L_i^-1
// (eq. Crack_approx_Fdot, D at level n), accumulated as
// M = sum_j V_j (1 - D_j)(v_j - v_i) (x) gradW_ij and dF/dt = M L_i^-1; then
// the constitutive update and Q_i = P_i L_i^-T (0 for failed particles).
// A neighbour as the deformation pass needs it: reference position,
// half-step velocity and V0 (1 - D).
struct NbrA {
    double x, y, z, vx, vy, vz, w;
    double hs;   // support radius (graded spacing only)
};

// Artificial viscosity of one specimen as the gather uses it: pair factor
// -Q1 c0 mu + Q2 mu^2 (Pi rho0) for approaching pairs, mu = h v_ij.X_ij /
// (|X_ij|^2 + 0.01 h^2).
template <typename R>
struct AvPar {
    R q1c0, q2, h, eh2;
    bool on;
};
template <typename R>
__device__ __forceinline__ AvPar<R> av_par(const DevSpec& P) {
    return AvPar<R>{R(P.av_q1 * P.c0), R(P.av_q2), R(P.h), R(0.01 * P.h * P.h),
                    P.av_q1 != 0.0 || P.av_q2 != 0.0};
}

// The first G groups of a particle's neighbour indices (neighbours below
// kGatherA G), loaded before the staging of the staged pass; its local slots
// are below 2^16, two to a register.
constexpr int kGatherA = 4;
template <int G>
struct PreIdxA {
    uint32_t w[G][kGatherA / 2];
    __device__ int at(int g, int t) const {
        return (int)((t & 1) ? w[g][t >> 1] >> 16 : w[g][t >> 1] & 0xffffu);
    }
};
template <int G, typename IdxOf>
__device__ __forceinline__ PreIdxA<G> pre_indices_a(int cnt, IdxOf idx) {
    PreIdxA<G> p;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int t = 0; t < kGatherA; t += 2) {
            const int k = g * kGatherA + t;
            p.w[g][t >> 1] = (uint32_t)idx(k < cnt ? k : 0) |
                             ((uint32_t)idx(k + 1 < cnt ? k + 1 : 0) << 16);
        }
    return p;
}

// One group of kGatherA neighbours of the deformation pass's sums (group
// start k0): record loads first, then the arithmetic.
template <typename R, bool kExt, bool kVarH, typename RecOf>
__device__ __forceinline__ void gather_group(const D4& xi, const D4& vi, int cnt, int k0, R inv_h,
                                             const int (&j)[kGatherA], RecOf rec, R M[9],
                                             const AvPar<R>& av, R AV[3], double hi) {
    NbrA nb[kGatherA];
#pragma unroll
    for (int t = 0; t < kGatherA; ++t) nb[t] = rec(j[t]);
#pragma unroll
    for (int t = 0; t < kGatherA; ++t) {
        // past the last neighbour 1/r = 0 makes every term an exact zero
        const bool live = k0 + t < cnt;
        const R dx = R(nb[t].x - xi.x), dy = R(nb[t].y - xi.y), dz = R(nb[t].z - xi.z);
        const R r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const R ir = live ? rsqrt_pos(r2) : R(0);
        R ih = inv_h, hpair = av.h;
        if constexpr (kVarH) {
            hpair = R(0.5 * (hi + nb[t].hs));
            ih = rcp_nr(hpair);
        }
        const R q = r2 * ir * ih;
        // h dW/dr / c = -6 (1 - q)^2 + 24 max(1/2 - q, 0)^2, no branch
        const R a = R(1) - q;
        const R b = fmax(R(0.5) - q, R(0));
        const R sl = fma(R(24), b * b, R(-6) * (a * a));
        R gw = sl * ir * R(nb[t].w);
        if constexpr (kVarH) gw *= R(8.0 / M_PI) * ih * ih * ih * ih;
        const R gx = gw * dx, gy = gw * dy, gz = gw * dz;
        const R t0 = R(nb[t].vx - vi.x), t1 = R(nb[t].vy - vi.y), t2 = R(nb[t].vz - vi.z);
        M[0] = fma(t0, gx, M[0]); M[1] = fma(t0, gy, M[1]); M[2] = fma(t0, gz, M[2]);
        M[3] = fma(t1, gx, M[3]); M[4] = fma(t1, gy, M[4]); M[5] = fma(t1, gz, M[5]);
        M[6] = fma(t2, gx, M[6]); M[7] = fma(t2, gy, M[7]); M[8] = fma(t2, gz, M[8]);
        if constexpr (kExt) {
            // sum_j (-Q1 c0 mu + Q2 mu^2) V_j (1 - D_j) gradW_ij over approaching pairs
            if (av.on) {
                const R vx = fma(t0, dx, fma(t1, dy, t2 * dz));
                if (vx < R(0)) {
                    const R eh2 = kVarH ? R(0.01) * hpair * hpair : av.eh2;
                    const R mu = hpair * vx * rcp_nr(r2 + eh2);
                    const R pi = mu * fma(av.q2, mu, -av.q1c0);
                    AV[0] = fma(pi, gx, AV[0]);
                    AV[1] = fma(pi, gy, AV[1]);
                    AV[2] = fma(pi, gz, AV[2]);
                }
            }
        }
    }
}

// M = sum_j V_j (1 - D_j)(v_j - v_i) (x) gradW_ij over the neighbours in
// increasing order, in groups of kGatherA whose record loads are all issued
// before their arithmetic: the first G groups from preloaded indices, the
// rest with indices one group ahead.  The kernel slope enters without its
// constant factor c / h (c = 8 / (pi h^3)), applied to the sum.  Graded
// spacing (kVarH): each pair has its own support h_ij = (h_i + h_j)/2 (h_i =
// hi), and the kernel's constant factor enters per pair (grad_k = 1).
template <typename R, bool kExt, bool kVarH = false, int G = 0, typename IdxOf, typename RecOf>
__device__ __forceinline__ void gather_fdot(const D4& xi, const D4& vi, int cnt, R inv_h, R grad_k,
                                            IdxOf idx, RecOf rec, R M[9], const AvPar<R>& av,
                                            R AV[3], double hi = 0.0,
                                            const PreIdxA<(G > 0 ? G : 1)>* pre = nullptr) {
#pragma unroll
    for (int q = 0; q < 9; ++q) M[q] = R(0);
    AV[0] = AV[1] = AV[2] = R(0);
    // the first group past the preloaded ones goes out first
    int jn[kGatherA];
#pragma unroll
    for (int t = 0; t < kGatherA; ++t) {
        const int k = G * kGatherA + t;
        jn[t] = idx(k < cnt ? k : 0);
    }
    if constexpr (G > 0) {
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (g * kGatherA < cnt) {
                int j[kGatherA];
#pragma unroll
                for (int t = 0; t < kGatherA; ++t) j[t] = pre->at(g, t);
                gather_group<R, kExt, kVarH>(xi, vi, cnt, g * kGatherA, inv_h, j, rec, M, av, AV,
                                             hi);
            }
    }
    for (int k0 = G * kGatherA; k0 < cnt; k0 += kGatherA) {
        int j[kGatherA];
#pragma unroll
        for (int t = 0; t < kGatherA; ++t) {
            j[t] = jn[t];
            const int kn = k0 + kGatherA + t;
            jn[t] = idx(kn < cnt ? kn : 0);
        }
        gather_group<R, kExt, kVarH>(xi, vi, cnt, k0, inv_h, j, rec, M, av, AV, hi);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) M[q] *= grad_k;
    if constexpr (kExt) {
        AV[0] *= grad_k; AV[1] *= grad_k; AV[2] *= grad_k;
    }
}

// The rest of the deformation pass for particle i (specimen sp) given M:
// dF/dt = M L_i^-1, the constitutive update, Q_i = P_i L_i^-T, stores.
// The first input of the particle's update, L^-1: the staged pass loads it
// before its neighbour sums, which then hide its latency (loading H^n and
// sigma^n there too would spill registers in the neighbour sums).
template <typename R>
struct UpdIn {
    R Li[9];
};
template <typename R>
__device__ __forceinline__ UpdIn<R> load_upd_in(const DevState& s, int64_t i) {
    const int64_t np = s.np;
    UpdIn<R> u;
    if constexpr (std::is_same<R, float>::value) {
#pragma unroll
        for (int k = 0; k < 9; ++k) u.Li[k] = s.Linv32[k * np + i];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) u.Li[k] = s.Linv[k * np + i];
    }
    return u;
}

template <typename R, int DM, bool kFlow>
__device__ __forceinline__ void pass_a_update(const DevState& s, int64_t i, int sp, const R M[9],
                                              double wi, const R AV[3], const UpdIn<R>& in) {
    const int64_t np = s.np;
    const DevSpec& P = s.specs[sp];
    R Li[9];
    R Fd[9];
    mm33(M, in.Li, Fd);
    GQRec<R>* __restrict__ GQ = gq_of<R>(s);
    GHRec<R>* __restrict__ GH = gh_of<R>(s);
    R Hn[9], sn[6];
    {
        const GHRec<R> gi = GH[i];
#pragma unroll
        for (int k = 0; k < 9; ++k) Hn[k] = gi.h[k];
    }
    if constexpr (std::is_same<R, float>::value) {
#pragma unroll
        for (int k = 0; k < 6; ++k) sn[k] = s.sig32[k * np + i];
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) sn[k] = s.sig[k * np + i];
    }
    double eps = s.eps_p[i], rate = s.eps_rate[i], e = s.e[i];
    const double rate0 = rate;
    double dinit = 0.0, wp = 0.0, fv = 0.0;
    const int model = DM >= 0 ? DM : P.damage;
    if (model == 1 || model == 2) dinit = s.d_init[i];
    if (model == 1) wp = s.w_p[i];
    if (model == 3) fv = s.f_void[i];
    const double Di = s.D[i];
    PointOut<R> o;
    int32_t flags = 0;
    point_update<R, DM, kFlow>(P, Hn, Fd, sn, eps, rate, dinit, wp, fv, e, Di, o, flags);
    // stores: the index passes through an empty asm so that store addresses
    // are formed here rather than kept in registers from the loads above
    int64_t is = i;
    asm volatile("" : "+v"(is));
    if constexpr (std::is_same<R, float>::value) {
#pragma unroll
        for (int k = 0; k < 6; ++k) s.sig32[k * np + is] = o.sig[k];
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) s.sig[k * np + is] = o.sig[k];
    }
    // L^-1 again (cached), rather than held in registers through the update
    if constexpr (std::is_same<R, float>::value) {
#pragma unroll
        for (int k = 0; k < 9; ++k) Li[k] = s.Linv32[k * np + is];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) Li[k] = s.Linv[k * np + is];
    }
    GQRec<R> go;
    GHRec<R> ho;
    const bool failed = o.D >= 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            go.q[3 * a + b] = failed ? R(0)
                                     : dot3(o.P[3 * a], Li[3 * b], o.P[3 * a + 1], Li[3 * b + 1],
                                            o.P[3 * a + 2], Li[3 * b + 2]);
#pragma unroll
    for (int k = 0; k < 9; ++k) ho.h[k] = o.H[k];
    go.omd = R(1.0 - o.D);
    ho.pad = R(0);
    GQ[is] = go;
    GH[is] = ho;
    // The plastic strain and its accumulators change only where the particle
    // yields (rate = increment / dt is then nonzero; a zero increment leaves
    // every one of them as it was), the rate also where it stops yielding, D
    // only where it grows: the other particles (most, in an elastic body)
    // store none of them, and memory lines holding no changed value are not
    // written.
    if (Di < 1.0) {
        s.e[is] = e;
        if (rate != 0.0) {
            s.eps_p[is] = eps;
            if (model == 1 || model == 2) s.d_init[is] = dinit;
            if (model == 1) s.w_p[is] = wp;
            if (model == 3) s.f_void[is] = fv;
        }
        if (rate != rate0) s.eps_rate[is] = rate;
    }
    if (o.D != Di) s.D[is] = o.D;
    if constexpr (kFlow) {
        // artificial viscous force for the next kick: rho0 V_i (1 - D_i) times
        // the gathered sum (w_i = V_i (1 - D_i^n))
        if (s.av) {
            const double k = P.rho0 * wi;
            s.fvisc[is] = k * double(AV[0]);
            s.fvisc[np + is] = k * double(AV[1]);
            s.fvisc[2 * np + is] = k * double(AV[2]);
        }
    }
    if (i == P.first) s.t[sp] += P.dt;
    if (flags || (s.flags & kFlagCheckFinite)) {
        int32_t fl = flags;
        if (s.flags & kFlagCheckFinite) {
            bool ok = true;
#pragma unroll
            for (int k = 0; k < 6; ++k) ok = ok && isfinite(double(o.sig[k]));
            if (!ok) fl |= kErrNonFinite;
        }
        if (fl) atomicOr(&s.err[2], fl);
    }
}

// Waves per SIMD the deformation pass is compiled for: three (at most 168
// registers) for each single damage model with Johnson-Cook hardening and
// the explicit return, and for the mixed form with the other flow laws (JC
// or no damage).  The FP64 GTN variant then spills 76 bytes (outside its
// Newton loops) and still runs faster than at two waves; the mixed-model
// variant and the FP64 form with the other flow laws would spill more and
// keep their registers.
template <typename R, int DM, bool kFlow>
__host__ __device__ constexpr int pass_a_waves_min() {
    return DM >= 0 && DM <= 3 && (!kFlow || (sizeof(R) == 4 && DM != 1)) ? 3 : 1;
}

// Specimen parameters are read with scalar loads: the lanes of a wave take
// turns by specimen, one turn unless the wave straddles two specimens.
template <typename R, int DM, bool kFlow, bool kVarH = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(pass_a_waves_min<R, DM, kFlow>(), 8)))
k_pass_a(DevState s, int /* displacement buffer: unused here */) {
    const int64_t i = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int sp_lane = s.spec[i];
    if (frozen(s, sp_lane)) return;
    for (;;) {
        const int sp = __builtin_amdgcn_readfirstlane(sp_lane);
        if (sp == sp_lane) {
            const DevSpec& P = s.specs[sp];
            const D4* __restrict__ XV = s.XV;
            const D4* __restrict__ VW = s.VW;
            const int32_t* __restrict__ cp = s.col + s.slice_ptr[i / kSlice] + (i % kSlice);
            R M[9], AV[3];
            const D4 vi = VW[i];
            gather_fdot<R, kFlow, kVarH>(XV[i], vi, s.nnb[i], R(P.inv_h),
                                         kVarH ? R(1) : R(P.grad_k),
                                         [&](int k) { return (int)cp[(int64_t)k * kSlice]; },
                                         [&](int j) {
                                             const D4 x = XV[j], v = VW[j];
                                             return NbrA{x.x, x.y, x.z, v.x, v.y, v.z, v.w,
                                                         kVarH ? s.hs[j] : 0.0};
                                         }, M, av_par<R>(P), AV, kVarH ? s.hs[i] : 0.0);
            pass_a_update<R, DM, kFlow>(s, i, sp, M, vi.w, AV, load_upd_in<R>(s, i));
            break;
        }
    }
}

// Neighbour-index groups the staged deformation pass loads before its
// staging.
template <typename R, int DM, bool kFlow>
__host__ __device__ constexpr int staged_a_pre_groups() {
    return sizeof(R) == 8 ? 6 : 3;
}

// The same pass over the force pass's tiles: the records of the tile and its
// halo (position, velocity, V0 (1 - D): 56 bytes) are staged in LDS once and
// the neighbour sums read them through the 16-bit local slots.  Same
// arithmetic in the same order as k_pass_a.
// Graded spacing (kVarH): the support radius follows (64 bytes).
constexpr int kLdsABytes = 56;
template <typename R, int DM, bool kFlow, bool kVarH = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(pass_a_waves_min<R, DM, kFlow>(), 8)))
k_pass_a_staged(DevState s, int /* displacement buffer: unused here */) {
    extern __shared__ __align__(16) unsigned char lds_a[];
    // G tiles per workgroup (two where a tile is not a whole number of waves),
    // each with an image of M slots of its own; thread tx of part `part`
    // takes particle tx of that part's tile
    const int M = s.lds_slots_a;
    const int T = s.tile_a;
    const int G = s.a_group;
    const int part = G > 1 ? (int)threadIdx.x / T : 0;
    const int tx = (int)threadIdx.x - part * T;
    const int64_t n_tiles = (s.n + T - 1) / T;
    const int32_t* cnt_a = s.run_count ? s.run_count + 3 : nullptr;
    if (work_tile(s.tile_list_a, cnt_a, G, 0, n_tiles) < 0) return;   // (then no part has a tile)
    const int64_t tile = work_tile(s.tile_list_a, cnt_a, G, part, n_tiles);
    const int64_t tl = tile < 0 ? 0 : tile;
    const size_t base = (size_t)part * M;
    const size_t GM = (size_t)G * M;
    double2* __restrict__ Lxy = reinterpret_cast<double2*>(lds_a) + base;
    double2* __restrict__ Lzw = reinterpret_cast<double2*>(lds_a) + GM + base;
    double2* __restrict__ Lvxy = reinterpret_cast<double2*>(lds_a) + 2 * GM + base;
    double* __restrict__ Lvz = reinterpret_cast<double*>(reinterpret_cast<double2*>(lds_a) + 3 * GM) + base;
    double* __restrict__ Lhs = reinterpret_cast<double*>(reinterpret_cast<double2*>(lds_a) + 3 * GM) + GM + base;
    const int64_t start = tl * T;
    const int32_t* __restrict__ hl = s.halo_a + tl * (int64_t)s.halo_cap_a;
    const D4* __restrict__ XV = s.XV;
    const D4* __restrict__ VW = s.VW;
    // Up to four slots per thread per round: index loads, record loads, LDS
    // stores (two memory latencies a round).  The first round's index loads
    // go out before the particle's own scalars, whose latency then overlaps
    // them; it needs no halo count (slots past the image hold n), which is
    // read after it.  Slots past the image, and past the particle count (last
    // tile), load the tile's first record and store nothing.
    constexpr int kU = 4;
    int m0 = tx;
    int64_t g[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) g[u] = slot_particle(m0 + u * T, T, s.halo_cap_a, start, s.n, hl);
    const int64_t i = start + tx;
    const bool in = tile >= 0 && i < s.n;
    const int64_t ii = in ? i : start;
    const int cnt = s.nnb[ii];
    const int64_t slice0 = s.slice_ptr[ii / kSlice];
    const int sp_lane = s.spec[ii];
    const uint16_t* __restrict__ lp = s.lcol_a + slice0 + (ii % kSlice);
    const auto idx = [&](int k) { return (int)lp[(int64_t)k * kSlice]; };
    constexpr int kPre = staged_a_pre_groups<R, DM, kFlow>();
    const PreIdxA<kPre> pre = pre_indices_a<kPre>(cnt, idx);
    // whether the specimen runs and (FP64: the mixed form has no registers to
    // spare for them) what the neighbour sums need of it: also loaded before
    // the staging
    constexpr bool kEarlyP = sizeof(R) == 8;
    const DevSpec& Pl = s.specs[sp_lane];
    const R inv_h_l = R(Pl.inv_h), grad_k_l = kVarH ? R(1) : R(Pl.grad_k);
    const AvPar<R> av_l = av_par<R>(Pl);
    const int32_t run_w = run_word(s, sp_lane);
    const auto stage = [&](int m0, const int64_t (&g)[kU]) {
        D4 x[kU], v[kU];
        double hv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t l = g[u] < s.n ? g[u] : start;
            x[u] = XV[l];
            v[u] = VW[l];
            if constexpr (kVarH) hv[u] = s.hs[l];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int m = m0 + u * T;
            if (g[u] < s.n) {
                Lxy[m] = double2{x[u].x, x[u].y};
                Lzw[m] = double2{x[u].z, v[u].w};
                Lvxy[m] = double2{v[u].x, v[u].y};
                Lvz[m] = v[u].z;
                if constexpr (kVarH) Lhs[m] = hv[u];
            }
        }
    };
    // (a part without a tile stages the first round of tile 0 into its own
    // image, which nothing reads: no branch holds the first round's loads back)
    stage(m0, g);
    const int tot = tile < 0 ? 0 : T + s.halo_cnt_a[tl];
    for (m0 += kU * T; m0 < tot; m0 += kU * T) {
#pragma unroll
        for (int u = 0; u < kU; ++u) g[u] = slot_particle(m0 + u * T, T, s.halo_cap_a, start, s.n, hl);
        stage(m0, g);
    }
    __syncthreads();
    if (!in || frozen_word(s, run_w)) return;
    const UpdIn<R> upd = load_upd_in<R>(s, i);
    for (;;) {
        const int sp = __builtin_amdgcn_readfirstlane(sp_lane);
        if (sp == sp_lane) {
            const DevSpec& P = s.specs[sp];
            const R inv_h = kEarlyP ? inv_h_l : R(P.inv_h);
            const R grad_k = kEarlyP ? grad_k_l : kVarH ? R(1) : R(P.grad_k);
            const AvPar<R> av = kEarlyP ? av_l : av_par<R>(P);
            const int t = tx;
            const double2 a = Lxy[t], b = Lzw[t], c = Lvxy[t];
            R M9[9], AV[3];
            gather_fdot<R, kFlow, kVarH, kPre>(
                D4{a.x, a.y, b.x, 0.0}, D4{c.x, c.y, Lvz[t], b.y}, cnt, inv_h, grad_k, idx,
                [&](int m) {
                    const double2 a = Lxy[m], b = Lzw[m], c = Lvxy[m];
                    return NbrA{a.x, a.y, b.x, c.x, c.y, Lvz[m], b.y, kVarH ? Lhs[m] : 0.0};
                },
                M9, av, AV, kVarH ? Lhs[t] : 0.0, &pre);
            pass_a_update<R, DM, kFlow>(s, i, sp, M9, b.y, AV, upd);
            break;
        }
    }
}

template <int S>
static hipError_t launch_b(const DevState& s, int parity, int block, bool mixed, hipStream_t st,
                           size_t lds_bytes) {
    if (s.staged) {
        const unsigned grid = (unsigned)((s.n + s.tile - 1) / s.tile);
        if (s.var_h) {   // graded spacing: per-pair supports
            if (mixed)
                k_pass_b_staged<float, S, true><<<grid, s.tile * S, lds_bytes, st>>>(s, parity);
            else
                k_pass_b_staged<double, S, true><<<grid, s.tile * S, lds_bytes, st>>>(s, parity);
        } else if (mixed) {
            k_pass_b_staged<float, S><<<grid, s.tile * S, lds_bytes, st>>>(s, parity);
        } else {
            k_pass_b_staged<double, S><<<grid, s.tile * S, lds_bytes, st>>>(s, parity);
        }
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)((s.n * S + block - 1) / block);
    if (s.var_h) {   // graded spacing: per-pair supports
        if (mixed)
            k_pass_b<float, S, true><<<grid, block, 0, st>>>(s, parity);
        else
            k_pass_b<double, S, true><<<grid, block, 0, st>>>(s, parity);
        return hipGetLastError();
    }
    if (mixed)
        k_pass_b<float, S><<<grid, block, 0, st>>>(s, parity);
    else
        k_pass_b<double, S><<<grid, block, 0, st>>>(s, parity);
    return hipGetLastError();
}

hipError_t launch_pass_b(const DevState& s, int parity, int block, int sub, bool mixed,
                         hipStream_t st, size_t lds_bytes) {
    if (!s.staged && (block <= 0 || block > 256 || block % sub != 0)) return hipErrorInvalidValue;
    switch (sub) {
        case 1: return launch_b<1>(s, parity, block, mixed, st, lds_bytes);
        case 2: return launch_b<2>(s, parity, block, mixed, st, lds_bytes);
        case 4: return launch_b<4>(s, parity, block, mixed, st, lds_bytes);
        default: return hipErrorInvalidValue;
    }
}

int staged_tile_max(int sub) { return staged_block_max(sub) / sub; }

size_t staged_record_bytes(bool mixed, bool var_h) {
    return 16 * (size_t)(mixed ? LdsB<float>::kUnits : LdsB<double>::kUnits) + (var_h ? 8 : 0);
}

size_t staged_a_record_bytes(bool var_h) { return kLdsABytes + (var_h ? 8 : 0); }

// Dynamic LDS above the default limit must be allowed per kernel.
hipError_t prepare_staged(size_t lds_bytes_b) {
    const void* fns[12] = {reinterpret_cast<const void*>(&k_pass_b_staged<double, 1>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<float, 1>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<double, 2>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<float, 2>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<double, 4>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<float, 4>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<double, 1, true>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<float, 1, true>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<double, 2, true>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<float, 2, true>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<double, 4, true>),
                           reinterpret_cast<const void*>(&k_pass_b_staged<float, 4, true>)};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes_b);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int DM, bool kFlow, bool kVarH = false>
static void launch_a(const DevState& s, int parity, unsigned grid, int block, bool mixed,
                     hipStream_t st) {
    if (block == 0) {   // staged over its tiles, a_group of them per workgroup
        const int64_t tiles = (s.n + s.tile_a - 1) / s.tile_a;
        const unsigned groups = (unsigned)((tiles + s.a_group - 1) / s.a_group);
        const int threads = s.tile_a * s.a_group;
        const size_t lds = (size_t)s.a_group * s.lds_slots_a * staged_a_record_bytes(kVarH);
        if (mixed)
            k_pass_a_staged<float, DM, kFlow, kVarH><<<groups, threads, lds, st>>>(s, parity);
        else
            k_pass_a_staged<double, DM, kFlow, kVarH><<<groups, threads, lds, st>>>(s, parity);
        return;
    }
    if (mixed)
        k_pass_a<float, DM, kFlow, kVarH><<<grid, block, 0, st>>>(s, parity);
    else
        k_pass_a<double, DM, kFlow, kVarH><<<grid, block, 0, st>>>(s, parity);
}

hipError_t launch_pass_a(const DevState& s, int parity, int block, bool mixed, hipStream_t st) {
    if (block == 0 && (!s.staged_lds_a || s.a_group < 1 || s.a_group > 2 ||
                       s.tile_a * s.a_group > 256))
        return hipErrorInvalidValue;
    const unsigned grid = block > 0 ? (unsigned)((s.n + block - 1) / block) : 0u;
    if (s.var_h) {   // graded spacing: the general variant with per-pair supports
        launch_a<-1, true, true>(s, parity, grid, block, mixed, st);
        return hipGetLastError();
    }
    if (s.flow_general) {
        switch (s.model) {
            case 0: launch_a<0, true>(s, parity, grid, block, mixed, st); break;
            case 1: launch_a<1, true>(s, parity, grid, block, mixed, st); break;
            case 2: launch_a<2, true>(s, parity, grid, block, mixed, st); break;
            case 3: launch_a<3, true>(s, parity, grid, block, mixed, st); break;
            default: launch_a<-1, true>(s, parity, grid, block, mixed, st); break;
        }
    } else {
        switch (s.model) {
            case 0: launch_a<0, false>(s, parity, grid, block, mixed, st); break;
            case 1: launch_a<1, false>(s, parity, grid, block, mixed, st); break;
            case 2: launch_a<2, false>(s, parity, grid, block, mixed, st); break;
            case 3: launch_a<3, false>(s, parity, grid, block, mixed, st); break;
            default: launch_a<-1, false>(s, parity, grid, block, mixed, st); break;
        }
    }
    return hipGetLastError();
}

// ===========================================================================
// field access in caller order
// ===========================================================================

enum Field {
    F_X = 0, F_U, F_V, F_DEFGRAD, F_SIGMA, F_EPS_P, F_EPS_P_RATE, F_D_INIT, F_W_P, F_VOID,
    F_D, F_E_INT, F_FORCE, F_Q, F_TIME, F_LINV, F_VISC, F_H
};

struct FieldRef {
    const double* d;   // double storage, or
    const float* f;    // float storage
    int comps;
    int kind;          // 0 plain, 1 deformation gradient stored as F - I, 2 damage
    int64_t cs, ps;    // element (particle p, component c) at [c * cs + p * ps]
};

__device__ __forceinline__ FieldRef field_ref(const DevState& s, int field, int par) {
    const int64_t np = s.np;
    switch (field) {
        case F_X: return {reinterpret_cast<const double*>(s.XV), nullptr, 3, 0, 1, 4};
        case F_U: return {reinterpret_cast<const double*>(s.U[par]), nullptr, 3, 0, 1, 4};
        case F_V: return {reinterpret_cast<const double*>(s.VW), nullptr, 3, 0, 1, 4};
        case F_DEFGRAD:
            return s.GH ? FieldRef{reinterpret_cast<const double*>(s.GH), nullptr, 9, 1, 1, 10}
                        : FieldRef{nullptr, reinterpret_cast<const float*>(s.GH32), 9, 1, 1, 10};
        case F_H:   // F - I as stored, without the round trip through F
            return s.GH ? FieldRef{reinterpret_cast<const double*>(s.GH), nullptr, 9, 0, 1, 10}
                        : FieldRef{nullptr, reinterpret_cast<const float*>(s.GH32), 9, 0, 1, 10};
        case F_Q:
            return s.GQ ? FieldRef{reinterpret_cast<const double*>(s.GQ), nullptr, 9, 0, 1, 10}
                        : FieldRef{nullptr, reinterpret_cast<const float*>(s.GQ32), 9, 0, 1, 10};
        case F_SIGMA:
            return s.sig ? FieldRef{s.sig, nullptr, 6, 0, np, 1} : FieldRef{nullptr, s.sig32, 6, 0, np, 1};
        case F_EPS_P: return {s.eps_p, nullptr, 1, 0, np, 1};
        case F_EPS_P_RATE: return {s.eps_rate, nullptr, 1, 0, np, 1};
        case F_D_INIT: return {s.d_init, nullptr, 1, 0, np, 1};
        case F_W_P: return {s.w_p, nullptr, 1, 0, np, 1};
        case F_VOID: return {s.f_void, nullptr, 1, 0, np, 1};
        case F_D: return {s.D, nullptr, 1, 2, np, 1};
        case F_E_INT: return {s.e, nullptr, 1, 0, np, 1};
        case F_FORCE: return {s.force, nullptr, 3, 0, np, 1};
        case F_LINV: return {s.Linv, nullptr, 9, 0, np, 1};
        case F_VISC: return {s.fvisc, nullptr, 3, 0, np, 1};
        default: return {nullptr, nullptr, 0, 0, 0, 0};
    }
}

__global__ void k_get(DevState s, int field, int par, double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const FieldRef r = field_ref(s, field, par);
    const int64_t p = s.iperm[i];
    for (int c = 0; c < r.comps; ++c) {
        const int64_t at = c * r.cs + p * r.ps;
        double x = r.d ? r.d[at] : (double)r.f[at];
        if (r.kind == 1 && (c % 4 == 0)) x += 1.0;
        dst[c * s.n + i] = x;
    }
}

// Writes keep the gathered copies consistent: damage also sets 1 - D in the
// force-pass record and V0 (1 - D) in the velocity record.
__global__ void k_set(DevState s, int field, int par, const double* __restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const FieldRef r = field_ref(s, field, par);
    const int64_t p = s.iperm[i];
    for (int c = 0; c < r.comps; ++c) {
        double x = src[c * s.n + i];
        if (r.kind == 1 && (c % 4 == 0)) x -= 1.0;
        const int64_t at = c * r.cs + p * r.ps;
        if (r.d)
            const_cast<double*>(r.d)[at] = x;
        else
            const_cast<float*>(r.f)[at] = (float)x;
    }
    if (r.kind == 2) {
        const double D = src[i];
        if (s.GQ) s.GQ[p].omd = 1.0 - D; else s.GQ32[p].omd = (float)(1.0 - D);
        s.VW[p].w = s.XV[p].w * (1.0 - D);
    }
}

hipError_t launch_get_field(const DevState& s, int field, int parity, bool, double* dst,
                            hipStream_t st) {
    const int T = 256;
    k_get<<<(unsigned)((s.n + T - 1) / T), T, 0, st>>>(s, field, parity, dst);
    return hipGetLastError();
}

hipError_t launch_set_field(const DevState& s, int field, int parity, bool, const double* src,
                            hipStream_t st) {
    const int T = 256;
    k_set<<<(unsigned)((s.n + T - 1) / T), T, 0, st>>>(s, field, parity, src);
    return hipGetLastError();
}

// ===========================================================================
// neighbour export (caller order, ascending rows)
// ===========================================================================

__global__ void k_export_count(DevState s, int64_t* __restrict__ row_ptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) row_ptr[0] = 0;
    if (i >= s.n) return;
    row_ptr[i + 1] = s.nnb[s.iperm[i]];
}

// in-place inclusive scan of a[0..m), one block
__global__ void __launch_bounds__(1024) k_scan_inplace(int64_t* __restrict__ a, int64_t m) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (m + 1023) / 1024;
    const int64_t lo = t * per, hi = (lo + per < m) ? lo + per : m;
    int64_t sum = 0;
    for (int64_t q = lo; q < hi; ++q) sum += a[q];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int q = 0; q < 1024; ++q) {
            const int64_t v = part[q];
            part[q] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t q = lo; q < hi; ++q) {
        run += a[q];
        a[q] = run;
    }
}

__global__ void k_export_fill(DevState s, const int64_t* __restrict__ row_ptr,
                              int32_t* __restrict__ col_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int64_t p = s.iperm[i];
    const int cnt = s.nnb[p];
    const int32_t* cp = s.col + s.slice_ptr[p / kSlice] + (p % kSlice);
    int32_t* out = col_out + row_ptr[i];
    for (int k = 0; k < cnt; ++k) {
        const int32_t v = s.perm[cp[(int64_t)k * kSlice]];
        int q = k;
        while (q > 0 && out[q - 1] > v) {
            out[q] = out[q - 1];
            --q;
        }
        out[q] = v;
    }
}

hipError_t launch_export_neighbors(const DevState& s, int64_t* row_ptr, int32_t* col, int64_t*,
                                   hipStream_t st) {
    const int T = 256;
    const unsigned g = (unsigned)((s.n + T - 1) / T);
    k_export_count<<<g, T, 0, st>>>(s, row_ptr);
    k_scan_inplace<<<1, 1024, 0, st>>>(row_ptr + 1, s.n);
    k_export_fill<<<g, T, 0, st>>>(s, row_ptr, col);
    return hipGetLastError();
}

// ===========================================================================
// diagnostics
// ===========================================================================

// members of each prescribed-velocity group, ordered by (group, sorted index)
__global__ void k_bc_keys(DevState s, uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                          int64_t n_pow2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pow2) return;
    const int g = (p < s.n) ? s.bc[p] : -1;
    keys[p] = g >= 0 ? (((uint64_t)g << 32) | (uint64_t)p) : ~0ull;
    vals[p] = (int32_t)p;
}

__global__ void k_bc_ptr(DevState s, const uint64_t* __restrict__ keys, int64_t n,
                         const int32_t* __restrict__ vals, int32_t* __restrict__ bc_list,
                         int64_t* __restrict__ bc_ptr) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= s.n_bc) {
        const uint64_t key = (uint64_t)t << 32;
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < key) lo = mid + 1; else hi = mid;
        }
        bc_ptr[t] = lo;
    }
    if (t < n && keys[t] != ~0ull) bc_list[t] = vals[t];
}

// ===========================================================================
// penalty contact: candidate lists from the current configuration
// ===========================================================================

// Bounding box of the current positions and the largest contact radius over
// every particle, in two stages: kCBoxParts workgroups each reduce a
// contiguous share of the particles to 7 partial extrema (lo[3], hi[3],
// max a) after the header, then one workgroup reduces those to the header:
// cbox = lo[3], hi[3], 1 / cell edge, cell edge (the edge 2 max a + skin, a
// hair larger), then the grid's extent in cells along x, y, z and whether
// the grid is dense (its cells fit the slot table, see CHash).  Minima and
// maxima do not depend on the order of reduction.
constexpr int kCBoxThreads = 256;

__device__ __forceinline__ void cbox_reduce(double (*red)[kCBoxThreads], double v[7]) {
    for (int a = 0; a < 7; ++a) red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int w = kCBoxThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 7; ++a) {
                const double o = red[a][threadIdx.x + w];
                red[a][threadIdx.x] = a < 3 ? fmin(red[a][threadIdx.x], o)
                                            : fmax(red[a][threadIdx.x], o);
            }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kCBoxThreads) k_cbox_part(DevState s, int par,
                                                             double* __restrict__ cbox) {
    __shared__ double red[7][kCBoxThreads];
    const D4* __restrict__ Uc = s.U[par];
    double v[7] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300, 0.0};
    const int64_t share = (s.n + kCBoxParts - 1) / kCBoxParts;
    const int64_t p0 = (int64_t)blockIdx.x * share;
    const int64_t p1 = p0 + share < s.n ? p0 + share : s.n;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += kCBoxThreads) {
        const D4 x = s.XV[p], u = Uc[p];
        const double c[3] = {x.x + u.x, x.y + u.y, x.z + u.z};
        for (int a = 0; a < 3; ++a) {
            v[a] = fmin(v[a], c[a]);
            v[3 + a] = fmax(v[3 + a], c[a]);
        }
        v[6] = fmax(v[6], s.arad[p]);
    }
    cbox_reduce(red, v);
    if (threadIdx.x < 7) cbox[kCBoxHead + (int64_t)blockIdx.x * 7 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kCBoxThreads) k_cbox_final(DevState s, double* __restrict__ cbox,
                                                              int64_t n_slots) {
    __shared__ double red[7][kCBoxThreads];
    double v[7] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300, 0.0};
    for (int b = threadIdx.x; b < kCBoxParts; b += kCBoxThreads)
        for (int a = 0; a < 7; ++a) {
            const double o = cbox[kCBoxHead + (int64_t)b * 7 + a];
            v[a] = a < 3 ? fmin(v[a], o) : fmax(v[a], o);
        }
    cbox_reduce(red, v);
    if (threadIdx.x < 6) cbox[threadIdx.x] = red[threadIdx.x][0];
    if (threadIdx.x == 0) {
        const double edge = (2.0 * red[6][0] + s.contact_skin) * (1.0 + 1e-9);
        const double inv = 1.0 / edge;
        cbox[6] = inv;
        cbox[7] = edge;
        // the cell of the largest coordinate, computed as every particle's
        // own (so no particle lies beyond it), bounds the extent
        double cells = 1.0;
        for (int a = 0; a < 3; ++a) {
            // (no finite position at all: an empty box, one cell)
            const double q = floor((red[3 + a][0] - red[a][0]) * inv);
            const double e = !(q >= 0.0) ? 1.0
                             : q >= (double)((1 << kCellBits) - 1) ? (double)(1 << kCellBits)
                                                                     : q + 1.0;
            cbox[9 + a] = e;
            cells *= e;
        }
        cbox[8] = cells <= (double)n_slots ? 1.0 : 0.0;
    }
}

__device__ __forceinline__ bool contact_cell(const double* cb, double x, double y, double z,
                                             int32_t c[3]) {
    constexpr double kLast = (double)((1 << kCellBits) - 1);
    const double xs[3] = {x, y, z};
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        const double q = floor((xs[a] - cb[a]) * cb[6]);
        // (a position that is not a number lands in cell 0 and is flagged)
        c[a] = !(q >= 0.0) ? 0 : (q >= kLast ? (1 << kCellBits) - 1 : (int32_t)q);
        if (!(q < kLast)) ok = false;
    }
    return ok;
}

// Packed key of a contact cell (coordinates below 2^kCellBits each).
__device__ __forceinline__ uint64_t ccell_key(const int32_t c[3]) {
    return (uint64_t)c[0] | ((uint64_t)c[1] << kCellBits) |
           ((uint64_t)c[2] << (2 * kCellBits));
}

// The grid as the rebuild's kernels read it from the bounding box: dense
// (slot = linear cell index, x fastest) or hashed, and its extent.
struct CGrid {
    bool dense;
    int32_t ext[3];
};
__device__ __forceinline__ CGrid cgrid(const double* cbox) {
    return CGrid{cbox[8] != 0.0, {(int32_t)cbox[9], (int32_t)cbox[10], (int32_t)cbox[11]}};
}
__device__ __forceinline__ int64_t cgrid_slot(const CGrid& g, int32_t x, int32_t y, int32_t z) {
    return ((int64_t)z * g.ext[1] + y) * g.ext[0] + x;
}

// First slot probed for a key (Fibonacci hashing), then linear probing.
__device__ __forceinline__ int64_t chash_home(const CHash& h, uint64_t key) {
    return (int64_t)((key * 0x9E3779B97F4A7C15ull) >> h.shift);
}

__global__ void k_chash_clear(CHash h) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= h.H) return;
    h.slot[t] = CSlot{~0ull, 0, 0};
}

// Each particle claims (or finds) its cell's slot and takes a place in the
// cell's group: rank[p] = slot << 32 | place (the place depends on the order
// of the atomics; the groups are put in index order afterwards).  Keys only
// ever go from empty to set, so particles of one cell, probing the same
// sequence, all stop at the same slot.
__global__ void k_chash_insert(DevState s, int par, const double* __restrict__ cbox, CHash h,
                               uint64_t* __restrict__ rank) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.n) return;
    const D4 x = s.XV[p], u = s.U[par][p];
    int32_t c[3];
    if (!contact_cell(cbox, x.x + u.x, x.y + u.y, x.z + u.z, c)) atomicOr(&s.err[2], kErrContact);
    const CGrid G = cgrid(cbox);
    int64_t t;
    if (G.dense) {
        // every cell lies inside the extent (the extent is the cell of the
        // largest coordinate, computed the same way); the clamp only keeps
        // the slot inside the table whatever the input
        for (int a = 0; a < 3; ++a) c[a] = c[a] < G.ext[a] ? c[a] : G.ext[a] - 1;
        t = cgrid_slot(G, c[0], c[1], c[2]);
    } else {
        const uint64_t key = ccell_key(c);
        t = chash_home(h, key);
        for (;;) {
            const unsigned long long old =
                atomicCAS((unsigned long long*)&h.slot[t].key, ~0ull, (unsigned long long)key);
            if (old == ~0ull || old == key) break;
            t = (t + 1) & (h.H - 1);
        }
    }
    const int32_t place = atomicAdd(&h.slot[t].cnt, 1);
    rank[p] = ((uint64_t)t << 32) | (uint32_t)place;
}

// Exclusive prefix sum of the slot counts, first within blocks of
// kCHashScanB slots (256 threads, 16 consecutive slots each) into the slots'
// start, each block's total into boff; then over the blocks
// (k_chash_scan_top).
__global__ void __launch_bounds__(256) k_chash_scan(CHash h) {
    constexpr int kPer = kCHashScanB / 256;
    __shared__ int32_t tot[256];
    const int64_t i0 = (int64_t)blockIdx.x * kCHashScanB + (int64_t)threadIdx.x * kPer;
    int32_t v[kPer];
    int32_t run = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int32_t c = (i0 + k < h.H) ? h.slot[i0 + k].cnt : 0;
        v[k] = run;
        run += c;
    }
    tot[threadIdx.x] = run;
    __syncthreads();
    // inclusive scan of the thread totals (Hillis-Steele)
    for (int d = 1; d < 256; d <<= 1) {
        const int32_t o = (int)threadIdx.x >= d ? tot[threadIdx.x - d] : 0;
        __syncthreads();
        tot[threadIdx.x] += o;
        __syncthreads();
    }
    const int32_t base = tot[threadIdx.x] - run;
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        if (i0 + k < h.H) h.slot[i0 + k].start = base + v[k];
    if (threadIdx.x == 255) h.boff[blockIdx.x] = tot[255];
}

__global__ void __launch_bounds__(1024) k_chash_scan_top(CHash h, int32_t n_blocks) {
    __shared__ int32_t tot[1024];
    int32_t carry = 0;
    for (int32_t b0 = 0; b0 < n_blocks; b0 += 1024) {
        const int32_t b = b0 + (int32_t)threadIdx.x;
        const int32_t mine = b < n_blocks ? h.boff[b] : 0;
        tot[threadIdx.x] = mine;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int32_t o = (int)threadIdx.x >= d ? tot[threadIdx.x - d] : 0;
            __syncthreads();
            tot[threadIdx.x] += o;
            __syncthreads();
        }
        if (b < n_blocks) h.boff[b] = carry + tot[threadIdx.x] - mine;
        carry += tot[1023];
        __syncthreads();
    }
}

__global__ void k_chash_scatter(DevState s, CHash h, const uint64_t* __restrict__ rank,
                                int32_t* __restrict__ members) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.n) return;
    const uint64_t r = rank[p];
    const int64_t t = (int64_t)(r >> 32);
    members[(int64_t)h.slot[t].start + h.boff[t / kCHashScanB] + (uint32_t)r] = (int32_t)p;
}

// Every slot's offset made global (so that in a dense grid the cells of a
// row along x are one contiguous range) and each group put in ascending
// particle index (insertion sort; a group holds a few particles).
__global__ void k_chash_order(CHash h, int32_t* __restrict__ members) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= h.H) return;
    const int32_t m = h.slot[t].cnt;
    const int32_t g0 = h.slot[t].start + h.boff[t / kCHashScanB];
    h.slot[t].start = g0;
    if (m < 2) return;
    int32_t* g = members + g0;
    for (int32_t i = 1; i < m; ++i) {
        const int32_t v = g[i];
        int32_t j = i - 1;
        while (j >= 0 && g[j] > v) {
            g[j + 1] = g[j];
            --j;
        }
        g[j + 1] = v;
    }
}

// Current position and contact radius, reference position and support
// radius of every particle, in grouped order.
__global__ void k_chash_gather(DevState s, int par, CHash h,
                               const int32_t* __restrict__ members) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s.n) return;
    const int32_t q = members[j];
    const D4 x = s.XV[q], u = s.U[par][q];
    h.gpos[j] = D4{x.x + u.x, x.y + u.y, x.z + u.z, s.arad[q]};
    h.gref[j] = D4{x.x, x.y, x.z, s.hs[q]};
}

// Candidates of particle p: particles q != p within a_p + a_q + skin, over
// the 27 cells around p (in z, y, x order, particles by index within a
// cell); bit 31 marks a reference neighbour of the same specimen, i.e. one
// inside the support in the reference configuration (the neighbour search's
// own test, with the same arithmetic, so the mark agrees with the complete
// reference lists).  More than kContactCap candidates: flagged, the rest
// dropped.
struct CFill {
    int64_t p, np;
    double px, py, pz, ap, skin;
    D4 xp;
    int64_t first, last;
    double h2, hp;
    bool var_h;
    int cnt;
};

// Test one particle q (current position and radius g, reference position
// and support radius at gref[src]) and append it when it is a candidate.
__device__ __forceinline__ void cfill_try(const DevState& s, const CHash& h, CFill& f,
                                          int32_t q, const D4& g, int64_t src) {
    if (q == f.p) return;
    const double d0 = g.x - f.px, d1 = g.y - f.py, d2 = g.z - f.pz;
    const double rr = f.ap + g.w + f.skin;
    if (!(d0 * d0 + d1 * d1 + d2 * d2 < rr * rr)) return;
    bool ref = false;
    if (q >= f.first && q < f.last) {
        const D4 xq = h.gref[src];
        const double e0 = xq.x - f.xp.x, e1 = xq.y - f.xp.y, e2 = xq.z - f.xp.z;
        const double r2 = e0 * e0 + e1 * e1 + e2 * e2;
        double lim = f.h2;
        if (f.var_h) {
            const double hpq = 0.5 * (f.hp + xq.w);
            lim = hpq * hpq;
        }
        ref = r2 < lim;
    }
    if (f.cnt < kContactCap)
        s.ccol[(int64_t)f.cnt * f.np + f.p] = (int32_t)((uint32_t)q | (ref ? 0x80000000u : 0u));
    ++f.cnt;
}

// The 27 cells of a hashed grid: the three cells of a row along x are
// looked up together.
__device__ void cfill_hashed(const DevState& s, const CHash& h, const int32_t* members,
                             const int32_t c[3], CFill& f) {
    constexpr int32_t kAxis = 1 << kCellBits;
    for (int row = 0; row < 9; ++row) {
        const int32_t cy = c[1] + row % 3 - 1, cz = c[2] + row / 3 - 1;
        if (cy < 0 || cz < 0 || cy >= kAxis || cz >= kAxis) continue;
        uint64_t key[3];
        int64_t t[3];
        CSlot r[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int32_t cc[3] = {c[0] + k - 1, cy, cz};
            key[k] = (cc[0] >= 0 && cc[0] < kAxis) ? ccell_key(cc) : ~0ull;
            t[k] = chash_home(h, key[k]);
            r[k] = h.slot[t[k]];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (key[k] == ~0ull) continue;
            while (r[k].key != key[k] && r[k].key != ~0ull) {
                t[k] = (t[k] + 1) & (h.H - 1);
                r[k] = h.slot[t[k]];
            }
            if (r[k].key != key[k]) continue;
            for (int32_t i = r[k].start, e = r[k].start + r[k].cnt; i < e; ++i)
                cfill_try(s, h, f, members[i], h.gpos[i], i);
        }
    }
}

// One thread per particle.  In a dense grid the three cells of each of the
// nine rows along x are one contiguous range of the grouped list; otherwise
// the cells are looked up in the hash table.
__global__ void k_cfill(DevState s, int par, const double* __restrict__ cbox, CHash h,
                        const int32_t* __restrict__ members) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = s.np;
    if (p >= np) return;
    if (p >= s.n) {
        s.ccnt[p] = 0;
        return;
    }
    CFill f;
    const D4 xp = s.XV[p], up = s.U[par][p];
    f.p = p;
    f.np = np;
    f.px = xp.x + up.x;
    f.py = xp.y + up.y;
    f.pz = xp.z + up.z;
    s.ubuild[p] = up.x;
    s.ubuild[np + p] = up.y;
    s.ubuild[2 * np + p] = up.z;
    f.ap = s.arad[p];
    f.skin = s.contact_skin;
    f.xp = xp;
    const DevSpec& P = s.specs[s.spec[p]];
    f.first = P.first;
    f.last = P.last;
    f.h2 = P.h2;
    f.hp = s.hs[p];
    f.var_h = s.var_h;
    f.cnt = 0;
    int32_t c[3];
    contact_cell(cbox, f.px, f.py, f.pz, c);
    const CGrid G = cgrid(cbox);
    if (G.dense) {
        for (int a = 0; a < 3; ++a) c[a] = c[a] < G.ext[a] ? c[a] : G.ext[a] - 1;
        // the nine rows' ranges first, then each row's particles four at a
        // time (their loads issued together)
        const int32_t x0 = c[0] > 0 ? c[0] - 1 : 0;
        const int32_t x1 = c[0] + 1 < G.ext[0] ? c[0] + 1 : G.ext[0] - 1;
        int32_t j0[9], j1[9];
#pragma unroll
        for (int row = 0; row < 9; ++row) {
            const int32_t cy = c[1] + row % 3 - 1, cz = c[2] + row / 3 - 1;
            j0[row] = j1[row] = 0;
            if (cy < 0 || cz < 0 || cy >= G.ext[1] || cz >= G.ext[2]) continue;
            j0[row] = h.slot[cgrid_slot(G, x0, cy, cz)].start;
            const CSlot r1 = h.slot[cgrid_slot(G, x1, cy, cz)];
            j1[row] = r1.start + r1.cnt;
        }
        for (int row = 0; row < 9; ++row)
            for (int32_t j = j0[row]; j < j1[row]; j += 4) {
                int32_t q[4];
                D4 g[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int32_t i = j + k < j1[row] ? j + k : j;
                    q[k] = members[i];
                    g[k] = h.gpos[i];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (j + k < j1[row]) cfill_try(s, h, f, q[k], g[k], j + k);
            }
    } else {
        cfill_hashed(s, h, members, c, f);
    }
    if (f.cnt > kContactCap) {
        atomicOr(&s.err[2], kErrContact);
        f.cnt = kContactCap;
    }
    s.ccnt[p] = f.cnt;
}

// The rebuild: bounding box and cell edge, the occupied cells' hash table
// with a counting sort of the particles by cell (ranks in keys, the grouped
// list in vals, grouped positions in gpos and gref), then the lists.
hipError_t launch_contact_build(const DevState& s, int parity, uint64_t* keys, int32_t* vals,
                                const CHash& h, double* cbox, hipStream_t st) {
    k_cbox_part<<<kCBoxParts, kCBoxThreads, 0, st>>>(s, parity, cbox);
    k_cbox_final<<<1, kCBoxThreads, 0, st>>>(s, cbox, h.H);
    constexpr int T = 256;
    const unsigned gh = (unsigned)((h.H + T - 1) / T), gn = (unsigned)((s.n + T - 1) / T);
    const int32_t n_blocks = (int32_t)((h.H + kCHashScanB - 1) / kCHashScanB);
    k_chash_clear<<<gh, T, 0, st>>>(h);
    k_chash_insert<<<gn, T, 0, st>>>(s, parity, cbox, h, keys);
    k_chash_scan<<<(unsigned)n_blocks, 256, 0, st>>>(h);
    k_chash_scan_top<<<1, 1024, 0, st>>>(h, n_blocks);
    k_chash_scatter<<<gn, T, 0, st>>>(s, h, keys, vals);
    k_chash_order<<<gh, T, 0, st>>>(h, vals);
    k_chash_gather<<<gn, T, 0, st>>>(s, parity, h, vals);
    k_cfill<<<(unsigned)((s.np + T - 1) / T), T, 0, st>>>(s, parity, cbox, h, vals);
    return hipGetLastError();
}

hipError_t launch_bc_lists(const DevState& s, uint64_t* keys, int32_t* vals, int64_t n_pow2,
                           int32_t* bc_list, int64_t* bc_ptr, hipStream_t st) {
    const int T = 256;
    const unsigned g = (unsigned)((n_pow2 + T - 1) / T);
    k_bc_keys<<<g, T, 0, st>>>(s, keys, vals, n_pow2);
    hipError_t e = launch_bitonic_sort(keys, vals, n_pow2, st);
    if (e != hipSuccess) return e;
    const int64_t m = (s.n > s.n_bc + 1) ? s.n : s.n_bc + 1;
    k_bc_ptr<<<(unsigned)((m + T - 1) / T), T, 0, st>>>(s, keys, s.n, vals, bc_list, bc_ptr);
    return hipGetLastError();
}

// ===========================================================================
// run control: specimens of a batch that stop on their own
// ===========================================================================

// One block per specimen, after a step that read U[par] and wrote U[par ^ 1]:
// count the step, sum the watched group's force component in a fixed order
// (each thread a strided share of the group's list, then a tree), update the
// running peak, and stop the specimen once failed or at its cap.  A specimen
// that stops gets its new displacement copied into the other buffer too, so
// that it stays put whichever buffer later steps read.
__global__ void __launch_bounds__(256) k_run_control(DevState s, int par, RunSpec* __restrict__ run,
                                                     const int32_t* __restrict__ bc_list,
                                                     const int64_t* __restrict__ bc_ptr) {
    __shared__ double red[256];
    __shared__ int32_t why_s;
    const int sp = blockIdx.x;
    if (s.done[sp] != kRunning) return;
    RunSpec& C = run[sp];
    const int g = C.group;
    double acc = 0.0;
    if (g >= 0) {
        const double* __restrict__ f = s.force + (int64_t)C.axis * s.np;
        for (int64_t k = bc_ptr[g] + threadIdx.x; k < bc_ptr[g + 1]; k += blockDim.x)
            acc += f[bc_list[k]];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t steps = C.steps + 1;
        C.steps = steps;
        int32_t why = kRunning;
        if (g >= 0) {
            const double r = C.sign * red[0];
            C.last = r;
            if (r > C.peak) C.peak = r;
            if (C.peak > 0.0 && C.peak >= C.min_peak && r < C.drop * C.peak) why = kStopFailed;
        }
        if (why == kRunning && C.cap > 0 && steps >= C.cap) why = kStopCap;
        why_s = why;
        if (why != kRunning) {
            s.done[sp] = why;
            atomicOr(&s.run_count[1], 1);
        }
    }
    __syncthreads();
    if (why_s == kRunning) return;
    const DevSpec& P = s.specs[sp];
    D4* __restrict__ dst = s.U[par];
    const D4* __restrict__ src = s.U[par ^ 1];
    for (int64_t i = P.first + threadIdx.x; i < P.last; i += blockDim.x) dst[i] = src[i];
}

// Append, in ascending order, the tiles of T particles (sorted order) that
// hold a running specimen's particle to `list`; returns their count (every
// thread).  Specimens are contiguous in sorted order, so a tile holds those
// from its first particle's to its last's.  One block of up to 1024 threads.
__device__ int64_t list_running_tiles(const DevState& s, int64_t n_tiles, int T,
                                      int32_t* __restrict__ list, int32_t* wave_cnt) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t base = 0;
    for (int64_t t0 = 0; t0 < n_tiles; t0 += blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        bool act = false;
        if (t < n_tiles) {
            const int64_t a = t * T;
            const int64_t b = (a + T < s.n ? a + T : s.n) - 1;
            for (int sp = s.spec[a]; sp <= s.spec[b] && !act; ++sp) act = s.done[sp] == kRunning;
        }
        const uint64_t m = __ballot(act);
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int64_t off = base, tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            off += w < wave ? wave_cnt[w] : 0;
            tot += wave_cnt[w];
        }
        if (act) list[off + __popcll(m & ((1ull << lane) - 1))] = (int32_t)t;
        base += tot;
        __syncthreads();
    }
    return base;
}

// The run-control tile lists of both passes (one when they share their
// tiles) and the number of running specimens.  One block; unless `force`, it
// returns at once when no specimen stopped since the last lists.
__global__ void __launch_bounds__(1024) k_tile_list(DevState s, int force) {
    __shared__ int32_t wave_cnt[16];
    __shared__ int32_t running;
    int32_t* __restrict__ cnt = s.run_count;
    if (!force && cnt[1] == 0) return;
    if (threadIdx.x == 0) running = 0;
    __syncthreads();
    const int64_t nb = list_running_tiles(s, (s.n + s.tile - 1) / s.tile, s.tile, s.tile_list,
                                          wave_cnt);
    int64_t na = nb;
    if (s.tile_list_a != s.tile_list)
        na = list_running_tiles(s, (s.n + s.tile_a - 1) / s.tile_a, s.tile_a, s.tile_list_a,
                                wave_cnt);
    int32_t mine = 0;
    for (int sp = threadIdx.x; sp < s.n_spec; sp += blockDim.x) mine += s.done[sp] == kRunning;
    if (mine) atomicAdd(&running, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt[0] = (int32_t)nb;
        cnt[1] = 0;
        cnt[2] = running;
        cnt[3] = (int32_t)na;
    }
}

hipError_t launch_run_control(const DevState& s, int parity, RunSpec* run, const int32_t* bc_list,
                              const int64_t* bc_ptr, hipStream_t st) {
    k_run_control<<<(unsigned)s.n_spec, 256, 0, st>>>(s, parity, run, bc_list, bc_ptr);
    return hipGetLastError();
}

hipError_t launch_tile_list(const DevState& s, int force, hipStream_t st) {
    k_tile_list<<<1, 1024, 0, st>>>(s, force);
    return hipGetLastError();
}

template <int NV>
__device__ __forceinline__ void block_reduce(double (*red)[256], double v[NV], const bool is_max[NV]) {
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < NV; ++q)
                red[q][threadIdx.x] = is_max[q] ? fmax(red[q][threadIdx.x], red[q][threadIdx.x + w])
                                                : red[q][threadIdx.x] + red[q][threadIdx.x + w];
        __syncthreads();
    }
}

__device__ __forceinline__ int find_segment(const int64_t* seg, int n_seg, int64_t b) {
    int lo = 0, hi = n_seg;   // seg[lo] <= b < seg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// One block per chunk of kDiagChunk particles of one segment.  Specimen
// partials: kinetic energy, internal energy, failed count, max D; group
// partials: force sum, displacement sum, count.
__global__ void __launch_bounds__(256) k_diag_part(DevState s, int par, const int32_t* __restrict__ list,
                                                   const int64_t* __restrict__ bc_ptr,
                                                   const int64_t* __restrict__ seg, int n_seg,
                                                   double* __restrict__ part) {
    __shared__ double red[7][256];
    const int64_t b = blockIdx.x;
    const int q = find_segment(seg, n_seg, b);
    const int64_t c = b - seg[q];
    const int64_t np = s.np;
    double* o = part + kNDiag * b;
    if (q < s.n_spec) {
        const DevSpec& P = s.specs[q];
        const int64_t beg = P.first + c * kDiagChunk;
        const int64_t end = beg + kDiagChunk < P.last ? beg + kDiagChunk : P.last;
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t p = beg + threadIdx.x; p < end; p += 256) {
            const double m = P.rho0 * s.XV[p].w;
            const D4 vv = s.VW[p];
            v[0] += 0.5 * m * (vv.x * vv.x + vv.y * vv.y + vv.z * vv.z);
            v[1] += m * s.e[p];
            const double D = s.D[p];
            v[2] += D >= 1.0 ? 1.0 : 0.0;
            v[3] = fmax(v[3], D);
        }
        const bool mx[4] = {false, false, false, true};
        block_reduce<4>(red, v, mx);
        if (threadIdx.x < kNDiag) o[threadIdx.x] = threadIdx.x < 4 ? red[threadIdx.x][0] : 0.0;
    } else {
        const int g = q - s.n_spec;
        const int64_t beg = bc_ptr[g] + c * kDiagChunk;
        const int64_t end = beg + kDiagChunk < bc_ptr[g + 1] ? beg + kDiagChunk : bc_ptr[g + 1];
        const D4* uc = s.U[par];
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int64_t k = beg + threadIdx.x; k < end; k += 256) {
            const int64_t p = list[k];
            for (int cc = 0; cc < 3; ++cc) v[cc] += s.force[cc * np + p];
            const D4 up = uc[p];
            v[3] += up.x; v[4] += up.y; v[5] += up.z;
            v[6] += 1.0;
        }
        const bool mx[7] = {false, false, false, false, false, false, false};
        block_reduce<7>(red, v, mx);
        if (threadIdx.x < kNDiag) o[threadIdx.x] = threadIdx.x < 7 ? red[threadIdx.x][0] : 0.0;
    }
}

// One block per segment: the chunk partials in a fixed order.
__global__ void __launch_bounds__(256) k_diag_final(DevState s, const int64_t* __restrict__ seg,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ spec_out,
                                                    double* __restrict__ bc_out) {
    __shared__ double red[7][256];
    const int q = blockIdx.x;
    const bool spec = q < s.n_spec;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = seg[q] + threadIdx.x; b < seg[q + 1]; b += 256) {
        const double* pp = part + kNDiag * b;
        for (int k = 0; k < 7; ++k) v[k] = (spec && k == 3) ? fmax(v[k], pp[k]) : v[k] + pp[k];
    }
    const bool mx_spec[7] = {false, false, false, true, false, false, false};
    const bool mx_bc[7] = {false, false, false, false, false, false, false};
    block_reduce<7>(red, v, spec ? mx_spec : mx_bc);
    if (threadIdx.x != 0) return;
    if (spec) {
        double* o = spec_out + kNDiag * q;
        o[0] = red[0][0]; o[1] = red[1][0]; o[2] = red[2][0]; o[3] = red[3][0];
        o[4] = s.t[q]; o[5] = 0.0; o[6] = 0.0; o[7] = 0.0;
    } else {
        double* o = bc_out + kNDiag * (q - s.n_spec);
        const double cnt = red[6][0];
        for (int c = 0; c < 3; ++c) {
            o[c] = red[c][0];
            o[3 + c] = cnt > 0 ? red[3 + c][0] / cnt : 0.0;
        }
        o[6] = cnt;
        o[7] = 0.0;
    }
}

// ===========================================================================
// scratch of the allocation-free diagnostics entry point
// ===========================================================================

// Chunk partials of tlsph_get_diagnostics_static: one array per device, held
// until the process ends.  Host code must not pass `scratch` itself to a
// kernel (on the host it names a stand-in, not device memory): scratch_ptr
// looks up each device's address once, with that device current.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_ptr(double** out) {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static double* addr[kMaxDev] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_diagnostics(const DevState& s, int parity, const int32_t* bc_list,
                              const int64_t* bc_ptr, const int64_t* seg, int32_t n_seg,
                              int64_t n_chunks, double* part, double* spec_diag, double* bc_diag,
                              hipStream_t st) {
    if (n_chunks <= 0 || n_seg <= 0) return hipErrorInvalidValue;
    k_diag_part<<<(unsigned)n_chunks, 256, 0, st>>>(s, parity, bc_list, bc_ptr, seg, n_seg, part);
    k_diag_final<<<(unsigned)n_seg, 256, 0, st>>>(s, seg, part, spec_diag, bc_diag);
    return hipGetLastError();
}

}  // namespace tlsph
