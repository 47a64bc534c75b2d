// Internal types shared by the host runtime and the kernels of libtlsph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tlsph {

constexpr int kSlice = 64;          // particles per slice of the sliced neighbour layout
constexpr int kMortonBits = 14;     // cells per axis < 2^14
constexpr int kSpecShift = 3 * kMortonBits;
constexpr int kNDiag = 8;          // doubles per diagnostics record

// Per-specimen parameters as the kernels read them (raw + derived).
struct DevSpec {
    double rho0, E, nu, c0, S_alpha, Gamma0;
    double A, B, n, C, eps_dot0;
    double Wcr, D1, D2, D3, D4, D5;
    double q1, q2, q3, f0, fN, eN, sN, fc, fF, k_omega;
    double h, dt, hg_alpha;
    double wall_n[3], wall_d;
    // derived on the host at create
    double G;          // shear modulus E / (2 (1 + nu))
    double inv_h;      // 1 / h
    double wnorm;      // 8 / (pi h^3): cubic-spline normalisation in 3D
    double h2;         // h * h (neighbour test, same rounding as a plain product)
    double inv_cell;   // 1 / cell edge, the edge a hair above h so that pairs closer
                       // than h never sit two cells apart after rounding
    int32_t damage;
    int32_t has_wall;
    int64_t first, last;   // sorted-order particle range [first, last)
};

struct DevBC {
    int32_t mask;
    int32_t pad_;
    double v_max[3];
    double tau;
    double grad[9];
};

// Device pointers of one context (all per-particle arrays in Morton order with
// stride np, a multiple of kSlice; component c of a field at [c * np + i]).
struct DevState {
    int64_t n, np;
    int32_t n_spec, n_bc;
    uint32_t flags;
    int32_t pad_;
    const double* X;
    const double* V0;
    const int32_t* spec;
    const int32_t* bc;
    const int32_t* perm;     // sorted -> caller
    const int32_t* iperm;    // caller -> sorted
    const int32_t* nnb;      // neighbour count
    const int64_t* slice_ptr;
    const int32_t* col;
    int64_t col_cap;         // entries of col (k_cap * np)
    const double* Linv;
    const float* Linv32;
    const DevSpec* specs;
    const DevBC* bcs;
    double* t;
    double* u[2];
    double* v;
    double* F;       // FP64 form
    float* H;        // mixed form: F - I
    double* sig;     // FP64 form, Voigt
    float* sig32;    // mixed form
    double* Q;       // FP64 form
    float* Q32;      // mixed form
    double* eps_p;
    double* eps_rate;
    double* d_init;
    double* w_p;
    double* f_void;
    double* e;
    double* D[2];
    double* force;
    int32_t* err;    // [0] first singular (sorted), [1] max count, [2] sticky flags,
                     // [3] build status
};

enum : uint32_t { kFlagStoreForce = 1u, kFlagGraphs = 2u, kFlagCheckFinite = 4u };
enum : int32_t { kErrNonFinite = 1, kErrNewton = 2 };

// launch helpers implemented in tlsph_kernels.hip
hipError_t launch_pass_b(const DevState& s, int parity, int block, bool mixed, hipStream_t st);
hipError_t launch_pass_a(const DevState& s, int parity, int block, bool mixed, hipStream_t st);

struct BuildBuffers {
    const double* X_in;      // caller order [3][n]
    const double* V0_in;
    const int32_t* bc_in;
    const int64_t* spec_off; // device copy [n_spec + 1]
    double* bbox;            // [n_spec][6]
    uint64_t* keys;          // [n_pow2]
    int32_t* vals;           // [n_pow2]
    int64_t n_pow2;
};

hipError_t launch_build_count(DevState& s, const BuildBuffers& b, hipStream_t st);
hipError_t launch_build_fill(DevState& s, const BuildBuffers& b, hipStream_t st);
hipError_t launch_shape_and_init(const DevState& s, bool mixed, hipStream_t st);
hipError_t launch_get_field(const DevState& s, int field, int parity, bool mixed, double* dst,
                            hipStream_t st);
hipError_t launch_set_field(const DevState& s, int field, int parity, bool mixed,
                            const double* src, hipStream_t st);
hipError_t launch_export_neighbors(const DevState& s, int64_t* row_ptr, int32_t* col,
                                   int64_t* scratch, hipStream_t st);
hipError_t launch_diagnostics(const DevState& s, int parity, const int32_t* bc_list,
                              const int64_t* bc_ptr, double* spec_diag, double* bc_diag,
                              hipStream_t st);
hipError_t launch_bc_lists(const DevState& s, uint64_t* keys, int32_t* vals, int64_t n_pow2,
                           int32_t* bc_list, int64_t* bc_ptr, hipStream_t st);

}  // namespace tlsph
