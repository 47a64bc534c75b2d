// HIP kernels of the TLSPH damage step for gfx950 (MI355X).
//
// Data layout (all per-particle arrays in Morton order, stride np, a multiple
// of 64): field component c of particle i at [c * np + i].  The neighbour
// list is "sliced": the 64 particles of slice s = i / 64 keep their k-th
// neighbour at col[slice_ptr[s] + 64 k + (i % 64)], so the 64 lanes of a
// wavefront read 64 consecutive indices per neighbour step.  One lane owns
// one particle and sums its neighbours in a fixed order: no floating-point
// atomics anywhere, results independent of the launch shape.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "tlsph_internal.h"
#include "tlsph_math.h"

namespace tlsph {

// ===========================================================================
// neighbour-list build (Sec. 2: S_i fixed in the reference configuration)
// ===========================================================================

__device__ __forceinline__ uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    uint64_t m = 0;
    for (int b = 0; b < kMortonBits; ++b) {
        m |= (uint64_t((x >> b) & 1u) << (3 * b)) | (uint64_t((y >> b) & 1u) << (3 * b + 1)) |
             (uint64_t((z >> b) & 1u) << (3 * b + 2));
    }
    return m;
}

// per-specimen bounding box (caller order, particles contiguous per specimen)
__global__ void k_bbox(const double* __restrict__ X, int64_t n, const int64_t* __restrict__ off,
                       double* __restrict__ bbox) {
    __shared__ double red[6][256];
    const int s = blockIdx.x;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = off[s] + threadIdx.x; i < off[s + 1]; i += blockDim.x)
        for (int c = 0; c < 3; ++c) {
            const double x = X[c * n + i];
            lo[c] = x < lo[c] ? x : lo[c];
            hi[c] = x > hi[c] ? x : hi[c];
        }
    for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = lo[c];
        red[3 + c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int c = 0; c < 3; ++c) {
                red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + w]);
                red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) bbox[6 * s + threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ int spec_of(const int64_t* off, int n_spec, int64_t i) {
    int lo = 0, hi = n_spec;  // largest s with off[s] <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void cell_of(const DevSpec& P, const double* bb, double x, double y,
                                        double z, int32_t c[3]) {
    const double xs[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        const double q = floor((xs[a] - bb[a]) * P.inv_cell);
        c[a] = q < 0.0 ? 0 : (int32_t)q;
    }
}

__global__ void k_keys(const double* __restrict__ X, int64_t n, int64_t n_pow2,
                       const int64_t* __restrict__ off, int n_spec, const DevSpec* __restrict__ specs,
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
    cell_of(specs[s], bbox + 6 * s, X[i], X[n + i], X[2 * n + i], c);
    if (c[0] >= (1 << kMortonBits) || c[1] >= (1 << kMortonBits) || c[2] >= (1 << kMortonBits))
        atomicOr(&err[3], 1);
    keys[i] = ((uint64_t)s << kSpecShift) | morton3(c[0], c[1], c[2]);
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
        specs_out[p] = (int32_t)(keys[p] >> kSpecShift);
    } else {
        perm[p] = -1;
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
    cell_of(P, bbox + 6 * sp, xi, yi, zi, c);
    int count = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int32_t cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= (1 << kMortonBits) ||
                    cy >= (1 << kMortonBits) || cz >= (1 << kMortonBits))
                    continue;
                const uint64_t key = ((uint64_t)sp << kSpecShift) | morton3(cx, cy, cz);
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
                    if (r2 < P.h2) visit(count++, (int32_t)q);
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
    if (p >= s.n) return;
    if (s.slice_ptr[s.np / kSlice] > cap_slots) return;  // capacity error reported by the host
    int32_t* base = col + s.slice_ptr[p / kSlice] + (p % kSlice);
    for_neighbours(s, keys, bbox, p, [&](int k, int32_t q) { base[(int64_t)k * kSlice] = q; });
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
        spline(r, P.inv_h, P.wnorm, W, dW);
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
    for (int c = 0; c < 3; ++c) s.force[c * np + p] = 0.0;
    if (s.GB) {
        GBRec<double> g;
        for (int k = 0; k < 9; ++k) { g.q[k] = 0.0; g.h[k] = 0.0; }
        g.omd = 1.0 - D0;
        g.pad = 0.0;
        s.GB[p] = g;
    } else {
        GBRec<float> g;
        for (int k = 0; k < 9; ++k) { g.q[k] = 0.0f; g.h[k] = 0.0f; }
        g.omd = (float)(1.0 - D0);
        g.pad = 0.0f;
        s.GB32[p] = g;
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
    k_bbox<<<s.n_spec, 256, 0, st>>>(b.X_in, s.n, b.spec_off, b.bbox);
    k_keys<<<(unsigned)((b.n_pow2 + T - 1) / T), T, 0, st>>>(b.X_in, s.n, b.n_pow2, b.spec_off,
                                                             s.n_spec, s.specs, b.bbox, b.keys,
                                                             b.vals, s.err);
    for (int64_t k = 2; k <= b.n_pow2; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            k_bitonic<<<(unsigned)((b.n_pow2 + T - 1) / T), T, 0, st>>>(b.keys, b.vals, b.n_pow2,
                                                                        j, k);
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

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Give XCD x a contiguous run of tiles instead, so the neighbour halos
// of Morton-adjacent tiles are shared through one L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nblk) {
    constexpr int64_t kXcd = 8;
    const int64_t q = nblk / kXcd, r = nblk % kXcd;
    const int64_t x = b % kXcd, k = b / kXcd;
    return x * q + (x < r ? x : r) + k;
}

template <typename R>
__device__ __forceinline__ const GBRec<R>* gb_of(const DevState& s);
template <>
__device__ __forceinline__ const GBRec<double>* gb_of<double>(const DevState& s) { return s.GB; }
template <>
__device__ __forceinline__ const GBRec<float>* gb_of<float>(const DevState& s) { return s.GB32; }

// Pass B (forces at t^n, kick, drift).  Nodal force of Sec. 3.1,
//   f_i = V_i sum_j V_j [(1 - D_j) Q_i + (1 - D_i) Q_j] gradW_ij,
// evaluated as V_i [Q_i a + (1 - D_i) b] with a = sum_j V_j (1 - D_j) gradW_ij
// and b = sum_j V_j Q_j gradW_ij, plus hourglass control: with the error
// vector e_ij = (F_i + F_j)/2 X_ij - x_ij and delta = e_ij . x_ij / |x_ij|,
//   f_i^HG = -alpha E (1 - D_i) V_i sum_j (1 - D_j) V_j W_ij delta / |X_ij|^2
//            x_ij / |x_ij|.
// Then v += dt f / m, prescribed velocities at t^{n+1/2}, D = 1 at rest,
// u^{n+1} = u^n + dt v (into the other displacement buffer), rigid wall, and
// the record (v, V0 (1 - D)) the deformation pass gathers.
template <typename R>
__global__ void __launch_bounds__(256) k_pass_b(DevState s, int par) {
    const int64_t i = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int64_t np = s.np;
    const int sp = s.spec[i];
    const DevSpec& P = s.specs[sp];
    const D4* __restrict__ XV = s.XV;
    const D4* __restrict__ Uc = s.U[par];
    const GBRec<R>* __restrict__ GB = gb_of<R>(s);
    const D4 xi = XV[i];
    const D4 ui = Uc[i];
    const GBRec<R> gi = GB[i];
    const double Di = s.D[i];
    const R inv_h = R(P.inv_h), wnorm = R(P.wnorm);
    R a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0, g0 = 0, g1 = 0, g2 = 0;
    const int cnt = s.nnb[i];
    const int32_t* __restrict__ cp = s.col + s.slice_ptr[i / kSlice] + (i % kSlice);
    for (int k = 0; k < cnt; ++k) {
        const int32_t j = cp[(int64_t)k * kSlice];
        const D4 xj = XV[j];
        const GBRec<R> gj = GB[j];
        const D4 uj = Uc[j];
        const R dx = R(xj.x - xi.x), dy = R(xj.y - xi.y), dz = R(xj.z - xi.z);
        const R r = sqrt(dx * dx + dy * dy + dz * dz);
        const R ir = R(1) / r;
        R W, dW;
        spline(r, inv_h, wnorm, W, dW);
        const R gs = dW * ir;
        const R gx = gs * dx, gy = gs * dy, gz = gs * dz;
        const R Vj = R(xj.w);
        const R wj = Vj * gj.omd;
        a0 += wj * gx; a1 += wj * gy; a2 += wj * gz;
        b0 += Vj * (gj.q[0] * gx + gj.q[1] * gy + gj.q[2] * gz);
        b1 += Vj * (gj.q[3] * gx + gj.q[4] * gy + gj.q[5] * gz);
        b2 += Vj * (gj.q[6] * gx + gj.q[7] * gy + gj.q[8] * gz);
        // hourglass
        const R du0 = R(uj.x - ui.x), du1 = R(uj.y - ui.y), du2 = R(uj.z - ui.z);
        const R x0 = dx + du0, x1 = dy + du1, x2 = dz + du2;
        const R irc = R(1) / sqrt(x0 * x0 + x1 * x1 + x2 * x2);
        const R e0 = R(0.5) * ((gi.h[0] + gj.h[0]) * dx + (gi.h[1] + gj.h[1]) * dy +
                               (gi.h[2] + gj.h[2]) * dz) - du0;
        const R e1 = R(0.5) * ((gi.h[3] + gj.h[3]) * dx + (gi.h[4] + gj.h[4]) * dy +
                               (gi.h[5] + gj.h[5]) * dz) - du1;
        const R e2 = R(0.5) * ((gi.h[6] + gj.h[6]) * dx + (gi.h[7] + gj.h[7]) * dy +
                               (gi.h[8] + gj.h[8]) * dz) - du2;
        const R delta = (e0 * x0 + e1 * x1 + e2 * x2) * irc;
        const R c = wj * W * delta * ir * ir * irc;
        g0 += c * x0; g1 += c * x1; g2 += c * x2;
    }
    const R omDi = R(1.0 - Di);
    const R hgk = R(-P.hg_alpha * P.E) * omDi;
    const double Vi = xi.w;
    const double f0 = Vi * double(gi.q[0] * a0 + gi.q[1] * a1 + gi.q[2] * a2 + omDi * b0 + hgk * g0);
    const double f1 = Vi * double(gi.q[3] * a0 + gi.q[4] * a1 + gi.q[5] * a2 + omDi * b1 + hgk * g1);
    const double f2 = Vi * double(gi.q[6] * a0 + gi.q[7] * a1 + gi.q[8] * a2 + omDi * b2 + hgk * g2);
    // kick
    const double dt = P.dt;
    const double m = P.rho0 * Vi;
    const D4 vo = s.VW[i];
    double v[3] = {vo.x, vo.y, vo.z};
    v[0] += dt * f0 / m;
    v[1] += dt * f1 / m;
    v[2] += dt * f2 / m;
    const int g = s.bc[i];
    if (g >= 0) {
        const DevBC& B = s.bcs[g];
        const double th = s.t[sp] + 0.5 * dt;
        const double ramp = B.tau > 0.0 ? 1.0 - exp(-th / B.tau) : 1.0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (B.mask & (1 << c))
                v[c] = B.v_max[c] * ramp + (B.grad[3 * c] * xi.x + B.grad[3 * c + 1] * xi.y +
                                            B.grad[3 * c + 2] * xi.z);
    }
    if (Di >= 1.0) v[0] = v[1] = v[2] = 0.0;
    double un[3] = {ui.x + dt * v[0], ui.y + dt * v[1], ui.z + dt * v[2]};
    if (P.has_wall) {
        const double xw[3] = {xi.x + un[0], xi.y + un[1], xi.z + un[2]};
        const double dn = xw[0] * P.wall_n[0] + xw[1] * P.wall_n[1] + xw[2] * P.wall_n[2] - P.wall_d;
        if (dn < 0.0) {
            un[0] = (xw[0] - dn * P.wall_n[0]) - xi.x;
            un[1] = (xw[1] - dn * P.wall_n[1]) - xi.y;
            un[2] = (xw[2] - dn * P.wall_n[2]) - xi.z;
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
        s.force[i] = f0; s.force[np + i] = f1; s.force[2 * np + i] = f2;
    }
}

// Pass A (deformation and constitutive update to t^{n+1}).
//   dF/dt_i = sum_j V_j (1 - D_j)(v_j - v_i) (x) gradW_ij L_i^-1
// (eq. Crack_approx_Fdot, D at level n), accumulated as
// M = sum_j V_j (1 - D_j)(v_j - v_i) (x) gradW_ij and dF/dt = M L_i^-1; then
// the constitutive update and Q_i = P_i L_i^-T (0 for failed particles).
template <typename R>
__global__ void __launch_bounds__(256) k_pass_a(DevState s, int par) {
    const int64_t i = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int64_t np = s.np;
    const int sp = s.spec[i];
    const DevSpec& P = s.specs[sp];
    const D4* __restrict__ XV = s.XV;
    const D4* __restrict__ VW = s.VW;
    const D4 xi = XV[i];
    const D4 vi = VW[i];
    const R inv_h = R(P.inv_h), wnorm = R(P.wnorm);
    R M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int cnt = s.nnb[i];
    const int32_t* __restrict__ cp = s.col + s.slice_ptr[i / kSlice] + (i % kSlice);
    for (int k = 0; k < cnt; ++k) {
        const int32_t j = cp[(int64_t)k * kSlice];
        const D4 xj = XV[j];
        const D4 vj = VW[j];
        const R dx = R(xj.x - xi.x), dy = R(xj.y - xi.y), dz = R(xj.z - xi.z);
        const R r = sqrt(dx * dx + dy * dy + dz * dz);
        R W, dW;
        spline(r, inv_h, wnorm, W, dW);
        const R gs = dW / r;
        const R gx = gs * dx, gy = gs * dy, gz = gs * dz;
        const R wj = R(vj.w);
        const R t0 = wj * R(vj.x - vi.x), t1 = wj * R(vj.y - vi.y), t2 = wj * R(vj.z - vi.z);
        M[0] += t0 * gx; M[1] += t0 * gy; M[2] += t0 * gz;
        M[3] += t1 * gx; M[4] += t1 * gy; M[5] += t1 * gz;
        M[6] += t2 * gx; M[7] += t2 * gy; M[8] += t2 * gz;
    }
    R Li[9];
    if constexpr (std::is_same<R, float>::value) {
#pragma unroll
        for (int k = 0; k < 9; ++k) Li[k] = s.Linv32[k * np + i];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) Li[k] = s.Linv[k * np + i];
    }
    R Fd[9];
    mm33(M, Li, Fd);
    GBRec<R>* __restrict__ GB = const_cast<GBRec<R>*>(gb_of<R>(s));
    R Hn[9], sn[6];
    {
        const GBRec<R> gi = GB[i];
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
    double dinit = 0.0, wp = 0.0, fv = 0.0;
    const int model = P.damage;
    if (model == 1 || model == 2) dinit = s.d_init[i];
    if (model == 1) wp = s.w_p[i];
    if (model == 3) fv = s.f_void[i];
    const double Di = s.D[i];
    PointOut<R> o;
    int32_t flags = 0;
    point_update<R>(P, Hn, Fd, sn, eps, rate, dinit, wp, fv, e, Di, o, flags);
    // stores
    if constexpr (std::is_same<R, float>::value) {
#pragma unroll
        for (int k = 0; k < 6; ++k) s.sig32[k * np + i] = o.sig[k];
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) s.sig[k * np + i] = o.sig[k];
    }
    GBRec<R> go;
    const bool failed = o.D >= 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            go.q[3 * a + b] = failed ? R(0)
                                     : o.P[3 * a] * Li[3 * b] + o.P[3 * a + 1] * Li[3 * b + 1] +
                                           o.P[3 * a + 2] * Li[3 * b + 2];
#pragma unroll
    for (int k = 0; k < 9; ++k) go.h[k] = o.H[k];
    go.omd = R(1.0 - o.D);
    go.pad = R(0);
    GB[i] = go;
    if (Di < 1.0) {
        s.eps_p[i] = eps;
        s.eps_rate[i] = rate;
        s.e[i] = e;
        if (model == 1 || model == 2) s.d_init[i] = dinit;
        if (model == 1) s.w_p[i] = wp;
        if (model == 3) s.f_void[i] = fv;
    }
    s.D[i] = o.D;
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

hipError_t launch_pass_b(const DevState& s, int parity, int block, bool mixed, hipStream_t st) {
    const unsigned grid = (unsigned)((s.n + block - 1) / block);
    if (mixed)
        k_pass_b<float><<<grid, block, 0, st>>>(s, parity);
    else
        k_pass_b<double><<<grid, block, 0, st>>>(s, parity);
    return hipGetLastError();
}

hipError_t launch_pass_a(const DevState& s, int parity, int block, bool mixed, hipStream_t st) {
    const unsigned grid = (unsigned)((s.n + block - 1) / block);
    if (mixed)
        k_pass_a<float><<<grid, block, 0, st>>>(s, parity);
    else
        k_pass_a<double><<<grid, block, 0, st>>>(s, parity);
    return hipGetLastError();
}

// ===========================================================================
// field access in caller order
// ===========================================================================

enum Field {
    F_X = 0, F_U, F_V, F_DEFGRAD, F_SIGMA, F_EPS_P, F_EPS_P_RATE, F_D_INIT, F_W_P, F_VOID,
    F_D, F_E_INT, F_FORCE, F_Q, F_TIME, F_LINV
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
            return s.GB ? FieldRef{reinterpret_cast<const double*>(s.GB) + 9, nullptr, 9, 1, 1, 20}
                        : FieldRef{nullptr, reinterpret_cast<const float*>(s.GB32) + 9, 9, 1, 1, 20};
        case F_Q:
            return s.GB ? FieldRef{reinterpret_cast<const double*>(s.GB), nullptr, 9, 0, 1, 20}
                        : FieldRef{nullptr, reinterpret_cast<const float*>(s.GB32), 9, 0, 1, 20};
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
        if (s.GB) s.GB[p].omd = 1.0 - D; else s.GB32[p].omd = (float)(1.0 - D);
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

hipError_t launch_bc_lists(const DevState& s, uint64_t* keys, int32_t* vals, int64_t n_pow2,
                           int32_t* bc_list, int64_t* bc_ptr, hipStream_t st) {
    const int T = 256;
    const unsigned g = (unsigned)((n_pow2 + T - 1) / T);
    k_bc_keys<<<g, T, 0, st>>>(s, keys, vals, n_pow2);
    for (int64_t k = 2; k <= n_pow2; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            k_bitonic<<<g, T, 0, st>>>(keys, vals, n_pow2, j, k);
    const int64_t m = (s.n > s.n_bc + 1) ? s.n : s.n_bc + 1;
    k_bc_ptr<<<(unsigned)((m + T - 1) / T), T, 0, st>>>(s, keys, s.n, vals, bc_list, bc_ptr);
    return hipGetLastError();
}

template <int NV>
__device__ __forceinline__ void block_reduce(double (*red)[256], double v[NV], const bool is_max[NV]) {
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < NV; ++q)
                red[q][threadIdx.x] = is_max[q] ? fmax(red[q][threadIdx.x], red[q][threadIdx.x + w])
                                                : red[q][threadIdx.x] + red[q][threadIdx.x + w];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_spec_diag(DevState s, int par, double* __restrict__ out) {
    __shared__ double red[4][256];
    const int sp = blockIdx.x;
    const DevSpec& P = s.specs[sp];
    const int64_t np = s.np;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = P.first + threadIdx.x; p < P.last; p += 256) {
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
    if (threadIdx.x == 0) {
        double* o = out + kNDiag * sp;
        o[0] = red[0][0]; o[1] = red[1][0]; o[2] = red[2][0]; o[3] = red[3][0];
        o[4] = s.t[sp]; o[5] = 0.0; o[6] = 0.0; o[7] = 0.0;
    }
}

__global__ void __launch_bounds__(256) k_bc_diag(DevState s, int par, const int32_t* __restrict__ list,
                                                 const int64_t* __restrict__ ptr,
                                                 double* __restrict__ out) {
    __shared__ double red[7][256];
    const int g = blockIdx.x;
    const int64_t np = s.np;
    const D4* uc = s.U[par];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t q = ptr[g] + threadIdx.x; q < ptr[g + 1]; q += 256) {
        const int64_t p = list[q];
        for (int c = 0; c < 3; ++c) v[c] += s.force[c * np + p];
        const D4 up = uc[p];
        v[3] += up.x; v[4] += up.y; v[5] += up.z;
        v[6] += 1.0;
    }
    const bool mx[7] = {false, false, false, false, false, false, false};
    block_reduce<7>(red, v, mx);
    if (threadIdx.x == 0) {
        double* o = out + kNDiag * g;
        const double cnt = red[6][0];
        for (int c = 0; c < 3; ++c) {
            o[c] = red[c][0];
            o[3 + c] = cnt > 0 ? red[3 + c][0] / cnt : 0.0;
        }
        o[6] = cnt;
        o[7] = 0.0;
    }
}

hipError_t launch_diagnostics(const DevState& s, int parity, const int32_t* bc_list,
                              const int64_t* bc_ptr, double* spec_diag, double* bc_diag,
                              hipStream_t st) {
    k_spec_diag<<<s.n_spec, 256, 0, st>>>(s, parity, spec_diag);
    if (bc_diag && s.n_bc > 0) k_bc_diag<<<s.n_bc, 256, 0, st>>>(s, parity, bc_list, bc_ptr, bc_diag);
    return hipGetLastError();
}

}  // namespace tlsph
