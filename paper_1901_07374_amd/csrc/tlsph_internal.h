// Internal types shared by the host runtime and the kernels of libtlsph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tlsph {

constexpr int kSlice = 64;          // particles per slice of the sliced neighbour layout
constexpr int kCellBits = 14;     // cells per axis < 2^14
constexpr int kSpecShift = 3 * kCellBits;
constexpr int kSub = 4;            // partial sums per particle in the force pass (canonical order)
constexpr int kNDiag = 8;          // doubles per diagnostics record
constexpr int kDiagChunk = 2048;   // particles per partial sum of the diagnostics
constexpr int kTile = 256;         // most particles per workgroup tile of the LDS-staged pass
// Halo-row entries past a tile's halo count that hold n (no particle): a
// staging round reads at most 1024 slots (two per thread of a 512-thread
// force pass, four per thread of a 256-particle deformation tile).
constexpr int kHaloPad = 1024;
constexpr int kHaloSortMax = 8192; // tile entries sorted in LDS at build (kTile * k_cap)
constexpr int kContactCap = 32;    // contact candidates per particle
constexpr int kCBoxParts = 512;    // workgroups of the contact bounding-box reduction
constexpr int kCBoxHead = 16;      // doubles of the contact grid header before the partials
// doubles of the static scratch array of the allocation-free diagnostics
// (1 MiB per device: 16384 chunk partials of kNDiag doubles)
constexpr int64_t kScratchDoubles = 1 << 17;

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
    double inv_dt, inv_rho0, inv_eps_dot0;
    double grad_k;     // wnorm / h: the kernel slope's constant factor
    double hg_k;       // -hg_alpha E wnorm: the hourglass force's constant factor
    double dt_rho0;    // dt / rho0: the kick per unit force density
    int32_t damage;
    int32_t has_wall;
    int32_t flow;              // strain-hardening law (tlsph_flow)
    int32_t implicit_return;   // 1: flow stress at the step's end in Algorithm 1
    double flow_e0, flow_beta; // Swift offset strain, Voce saturation rate
    double av_q1, av_q2;       // artificial viscosity coefficients (0: off)
    double h_per_spacing;      // > 0: per-particle support h_i = this V_i^(1/3)
    double contact_k;          // penalty contact factor (0: off)
    double contact_comp;       // (1 - nu^2) / E: the specimen's share of 1 / E*
    int32_t newton_gtn;        // iteration caps: Algorithm 2's loops, the implicit return
    int32_t newton_impl;
    int64_t first, last;   // sorted-order particle range [first, last)
};

// Run control of a batch whose specimens stop on their own, per specimen:
// at a step cap, or once failed.  Failure is read off the specimen's load, as
// the tensile tests of Sec. 6 read the strain at failure off the decay of the
// stress after damage sets in: the load is the reaction of one boundary group
// (the sign-adjusted sum of one component of its particles' nodal forces),
// and the specimen has failed once it has fallen below `drop` times its
// running peak, after that peak reached `min_peak`.
struct RunSpec {
    int64_t cap;        // steps after which the specimen stops (0: no cap)
    int64_t steps;      // steps taken since the control was set
    double sign;        // reaction = sign * sum of the group's force component
    double drop;
    double min_peak;
    double peak;        // running peak of the reaction
    double last;        // reaction of the last step
    int32_t group;      // watched boundary group (-1: none)
    int32_t axis;       // its force component
};
enum : int32_t { kRunning = 0, kStopCap = 1, kStopFailed = 2 };

struct DevBC {
    int32_t mask;
    int32_t pad_;
    double v_max[3];
    double tau;
    double grad[9];
};

// Records read through neighbour gathers (array-of-structures, 16-byte
// aligned so a record arrives in a few 128-bit loads).
struct alignas(16) D4 {
    double x, y, z, w;
};

// What the force pass gathers from a neighbour besides geometry, in two
// records so that the deformation pass reads only H: Q = P L^-T with 1 - D,
// and H = F - I.  R is the storage precision (double, or float in the mixed
// form); each record is 10 values, aligned to two.
template <typename R>
struct alignas(2 * sizeof(R)) GQRec {
    R q[9];
    R omd;
};
template <typename R>
struct alignas(2 * sizeof(R)) GHRec {
    R h[9];
    R pad;
};

// Device pointers of one context.  Per-particle data is in Hilbert order;
// SoA fields have stride np (a multiple of kSlice), component c of particle
// i at [c * np + i]; AoS records are indexed by particle.
struct DevState {
    int64_t n, np;
    int32_t n_spec, n_bc;
    uint32_t flags;
    int32_t pad_;
    const D4* XV;            // reference position and volume (x, y, z, V0)
    const int32_t* spec;
    const int32_t* bc;
    const int32_t* perm;     // sorted -> caller
    const int32_t* iperm;    // caller -> sorted
    const int32_t* nnb;      // neighbour count
    const int64_t* slice_ptr;
    const int32_t* col;
    int64_t col_cap;         // entries of col (k_cap * np)
    const double* Linv;      // SoA [9][np]
    const float* Linv32;     // mixed form copy
    const DevSpec* specs;
    const DevBC* bcs;
    double* t;
    D4* U[2];                // displacement (x, y, z, 0), two buffers
    D4* VW;                  // half-step velocity and V0 (1 - D) (x, y, z, w)
    GQRec<double>* GQ;       // FP64 form
    GHRec<double>* GH;
    GQRec<float>* GQ32;      // mixed form
    GHRec<float>* GH32;
    double* sig;             // FP64 form, SoA Voigt
    float* sig32;            // mixed form
    double* eps_p;
    double* eps_rate;
    double* d_init;
    double* w_p;
    double* f_void;
    double* e;
    double* D;
    double* force;           // SoA [3][np]
    double* fvisc;           // SoA [3][np] artificial viscous force for the next kick
    double* hs;              // [np] support radius of each particle (build)
    double* arad;            // [np] contact radius V_i^(1/3) / 2 (build)
    int32_t* ccnt;           // [np] contact candidates
    int32_t* ccol;           // [kContactCap][np] candidate (sorted index, bit 31: a
                             // reference neighbour of the same specimen)
    double* ubuild;          // [3][np] displacement when the list was built
    double contact_skin;     // skin of the candidate list
    int32_t* err;    // [0] first singular (sorted), [1] max count, [2] sticky flags,
                     // [3] build status, [4] largest tile halo
    // LDS staging: per tile of `tile` particles, the sorted outside neighbours
    // (halo) and every neighbour as a local slot (tile member j - start, or
    // tile + position in the halo), in the sliced layout of col
    const int32_t* halo;      // [n_tiles][halo_cap]
    const int32_t* halo_cnt;  // [n_tiles]
    const uint16_t* lcol;
    int32_t halo_cap;
    int32_t staged;           // 1 when the staged force pass is in use
    int32_t lds_slots;        // record slots of the staged kernels' LDS images (tile + largest halo)
    int32_t model;            // damage model shared by every specimen, -1 if they differ
    int32_t flow_general;     // 1 if a specimen uses another law than JC, the implicit
                              // return or the artificial viscosity
    int32_t av;               // 1 if a specimen uses the artificial viscosity
    int32_t var_h;            // 1 if a specimen has graded spacing (per-particle support)
    int32_t contact;          // 1 if a specimen has penalty contact
    int32_t tile;             // particles per tile of the staged force pass (<= kTile)
    // The staged deformation pass's tiles: the force pass's (the same
    // arrays), or a size of their own (arrays of their own).
    int32_t staged_lds_a;     // 1 when the tile records of the deformation pass fit LDS
    int32_t a_group;          // tiles per workgroup of the staged deformation pass (1, 2)
    int32_t tile_a;           // its particles per tile
    int32_t halo_cap_a;
    int32_t lds_slots_a;      // slots of one tile's image
    int32_t pad3_;
    const int32_t* halo_a;
    const int32_t* halo_cnt_a;
    const uint16_t* lcol_a;
    // run control (all null when off): why each specimen stopped (kRunning
    // while it runs), the tiles of `tile` particles holding a running
    // specimen's particle (ascending), the same for tiles of `tile_a` (the
    // same list when the passes share their tiles), and [0] the force
    // pass's count, [1] nonzero once a specimen stopped after the lists were
    // made, [2] running specimens, [3] the deformation pass's count
    int32_t* done;
    int32_t* tile_list;
    int32_t* tile_list_a;
    int32_t* run_count;
};

enum : uint32_t { kFlagStoreForce = 1u, kFlagGraphs = 2u, kFlagCheckFinite = 4u,
                  kFlagNoStaging = 8u };
enum : int32_t { kErrNonFinite = 1, kErrNewton = 2, kErrContact = 4 };

// launch helpers implemented in tlsph_kernels.hip
// Deformation pass: `block` threads per workgroup, or 0 for the variant staged
// over the force pass's tiles (s.staged_lds_a must be set).
// Force pass: `sub` lanes per particle (1, 2 or 4); the unstaged variant runs
// `block` threads per workgroup, the LDS-staged one tile * sub.
hipError_t launch_pass_b(const DevState& s, int parity, int block, int sub, bool mixed,
                         hipStream_t st, size_t lds_bytes = 0);
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
// Halo lists and local slots for tiles of T particles (halo_cap = T k_cap)
// into the given arrays; the largest halo is max-reduced into s.err[4].
hipError_t launch_halo(const DevState& s, int k_cap, int T, int32_t* halo, int32_t* halo_cnt,
                       uint16_t* lcol, hipStream_t st);
hipError_t prepare_staged(size_t lds_bytes_b);
// Largest tile the staged force pass runs with `sub` lanes per particle.
int staged_tile_max(int sub);
// LDS bytes per slot of the staged force pass and the staged deformation pass
// (graded spacing adds the slot's support radius).
size_t staged_record_bytes(bool mixed, bool var_h);
size_t staged_a_record_bytes(bool var_h);
hipError_t launch_shape_and_init(const DevState& s, bool mixed, hipStream_t st);
hipError_t launch_get_field(const DevState& s, int field, int parity, bool mixed, double* dst,
                            hipStream_t st);
hipError_t launch_set_field(const DevState& s, int field, int parity, bool mixed,
                            const double* src, hipStream_t st);
hipError_t launch_export_neighbors(const DevState& s, int64_t* row_ptr, int32_t* col,
                                   int64_t* scratch, hipStream_t st);
// Two-level fixed-order reductions: chunk partials (seg[q] .. seg[q+1] are the
// chunks of segment q: specimens first, then boundary groups), then one block
// per segment.
// Device address of this device's static scratch array (kScratchDoubles
// doubles), looked up on the first call with the device current.
hipError_t scratch_ptr(double** out);
hipError_t launch_diagnostics(const DevState& s, int parity, const int32_t* bc_list,
                              const int64_t* bc_ptr, const int64_t* seg, int32_t n_seg,
                              int64_t n_chunks, double* part, double* spec_diag, double* bc_diag,
                              hipStream_t st);
// Cell table of the contact grid: H = 2 n_pow2 slots, each the count of a
// cell's particles and the offset of its group in the cell-grouped particle
// list (first within its scan block of kCHashScanB slots, then, once boff
// holds the blocks' offsets, the global offset).  A grid of at most H cells
// is dense: slot = linear cell index, x fastest, so that the groups follow
// the cells' order in space.  A larger grid hashes its occupied cells
// (open addressing, linear probing; at most n_pow2 occupied, so at least
// half the slots stay empty), the slot holding the packed cell key (~0 when
// empty).  The grouped list holds each cell's particles in ascending
// index order, with their current positions and contact radii, and their
// reference positions and support radii, beside them.
constexpr int kCHashScanB = 4096;
struct CSlot {
    uint64_t key;
    int32_t cnt;
    int32_t start;
};
struct CHash {
    CSlot* slot;      // [H]
    int32_t* boff;    // [H / kCHashScanB + 1]
    D4* gpos;         // [n_pow2] grouped x + u and contact radius
    D4* gref;         // [n_pow2] grouped X and support radius h
    int64_t H;
    int shift;        // 64 - log2 H
};
// Contact candidate lists from the current configuration (keys, vals: n_pow2
// scratch; cbox: kCBoxHead doubles of grid header, then kCBoxParts * 7
// doubles of partial extrema).
hipError_t launch_contact_build(const DevState& s, int parity, uint64_t* keys, int32_t* vals,
                                const CHash& h, double* cbox, hipStream_t st);
// Run control after a step of parity `parity`: count it, watch each running
// specimen's reaction, stop specimens (their displacement into both buffers),
// then remake the tile list if a specimen stopped (or always with `force`).
hipError_t launch_run_control(const DevState& s, int parity, RunSpec* run, const int32_t* bc_list,
                              const int64_t* bc_ptr, hipStream_t st);
hipError_t launch_tile_list(const DevState& s, int force, hipStream_t st);
hipError_t launch_bc_lists(const DevState& s, uint64_t* keys, int32_t* vals, int64_t n_pow2,
                           int32_t* bc_list, int64_t* bc_ptr, hipStream_t st);

}  // namespace tlsph
