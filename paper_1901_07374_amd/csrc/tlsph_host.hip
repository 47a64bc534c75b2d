// Host runtime of libtlsph: the C ABI declared in include/tlsph.h.
//
// The context owns host metadata only.  Every device array lives in the
// caller's workspace, carved here at 256-byte alignment; the library never
// allocates device memory, so tlsph_step enqueues nothing but kernels (and,
// with TLSPH_USE_GRAPHS, replays of a captured two-step graph).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/tlsph.h"
#include "tlsph_internal.h"

using namespace tlsph;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int64_t next_pow2(int64_t x) {
    int64_t p = 64;
    while (p < x) p <<= 1;
    return p;
}

// Offsets of every device array inside the workspace.
struct Layout {
    int64_t n, np, n_pow2, n_slices;
    int32_t n_spec, n_bc, k_cap;
    bool mixed;
    size_t XV, spec, bc, perm, iperm, nnb, slice_ptr, col, lcol, halo, halo_cnt, Linv, Linv32,
        specs, bcs, t;
    int64_t n_tiles;
    size_t GQ, GH, U0, U1, VW, sig, eps_p, eps_rate, d_init, w_p, f_void, e, D, force, fvisc, hs, err,
        arad, ccnt, ccol, ubuild, cbox, hslot, hboff, gpos, gref,
        spec_off, bbox, keys, vals, bc_list, bc_ptr, diag_seg, diag_part, backup,
        run, done, tile_list, run_count, halo_a, halo_cnt_a, lcol_a, tile_list_a;
    int64_t diag_chunk_cap;
    size_t state_begin, backup_bytes;
    size_t total;
};

Layout make_layout(int64_t n, int32_t n_spec, int32_t n_bc, int32_t k_cap, bool mixed) {
    Layout L{};
    L.n = n;
    L.np = (n + kSlice - 1) / kSlice * kSlice;
    L.n_pow2 = next_pow2(n);
    L.n_slices = L.np / kSlice;
    L.n_spec = n_spec;
    L.n_bc = n_bc;
    L.k_cap = k_cap;
    L.mixed = mixed;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        const size_t o = align_up(cur);
        cur = o + bytes;
        return o;
    };
    const size_t np = (size_t)L.np;
    L.XV = take(np * sizeof(D4));
    L.spec = take(np * 4);
    L.bc = take(np * 4);
    L.perm = take(np * 4);
    L.iperm = take((size_t)n * 4);
    L.nnb = take(np * 4);
    L.slice_ptr = take(((size_t)L.n_slices + 1) * 8);
    L.col = take((size_t)k_cap * np * 4);
    L.lcol = take((size_t)k_cap * np * 2);
    // staged-pass tiles hold 64..kTile particles (chosen at build): room for
    // ceil(n / T) tiles of T * k_cap halo entries at any such T
    L.n_tiles = (n + 63) / 64;
    L.halo = take(((size_t)n + kTile) * k_cap * 4);
    L.halo_cnt = take((size_t)L.n_tiles * 4);
    L.Linv = take(9 * np * 8);
    L.hs = take(np * 8);
    L.arad = take(np * 8);
    // contact candidate lists (rebuilt from the state, so outside the saved region)
    L.ccnt = take(np * 4);
    L.ccol = take((size_t)kContactCap * np * 4);
    L.ubuild = take(3 * np * 8);
    L.cbox = take((kCBoxHead + (size_t)kCBoxParts * 7) * 8);
    const size_t H = 2 * (size_t)L.n_pow2;
    L.hslot = take(H * sizeof(CSlot));
    L.hboff = take((H / kCHashScanB + 1) * 4);
    L.gpos = take((size_t)L.n_pow2 * sizeof(D4));
    L.gref = take((size_t)L.n_pow2 * sizeof(D4));
    L.Linv32 = take(mixed ? 9 * np * 4 : 0);
    L.specs = take((size_t)n_spec * sizeof(DevSpec));
    L.bcs = take((size_t)(n_bc > 0 ? n_bc : 1) * sizeof(DevBC));
    L.t = take((size_t)n_spec * 8);
    // evolving state, contiguous (saved and restored by the autotuner)
    L.state_begin = align_up(cur);
    L.GQ = take(np * (mixed ? sizeof(GQRec<float>) : sizeof(GQRec<double>)));
    L.GH = take(np * (mixed ? sizeof(GHRec<float>) : sizeof(GHRec<double>)));
    L.U0 = take(np * sizeof(D4));
    L.U1 = take(np * sizeof(D4));
    L.VW = take(np * sizeof(D4));
    L.sig = take(6 * np * (mixed ? 4 : 8));
    L.eps_p = take(np * 8);
    L.eps_rate = take(np * 8);
    L.d_init = take(np * 8);
    L.w_p = take(np * 8);
    L.f_void = take(np * 8);
    L.e = take(np * 8);
    L.D = take(np * 8);
    L.force = take(3 * np * 8);
    L.fvisc = take(3 * np * 8);
    L.backup_bytes = align_up(cur) - L.state_begin;
    L.err = take(8 * 4);
    L.spec_off = take(((size_t)n_spec + 1) * 8);
    L.bbox = take((size_t)n_spec * 8 * 8);
    L.keys = take((size_t)L.n_pow2 * 8);
    L.vals = take((size_t)L.n_pow2 * 4);
    L.bc_list = take(np * 4);
    L.bc_ptr = take(((size_t)n_bc + 2) * 8);
    // diagnostics partials: sum over segments of ceil(size / chunk), at most
    // 2 n / chunk + one per segment
    L.diag_chunk_cap = 2 * (n / kDiagChunk) + n_spec + n_bc + 2;
    L.diag_seg = take(((size_t)n_spec + n_bc + 1) * 8);
    L.diag_part = take((size_t)L.diag_chunk_cap * kNDiag * 8);
    L.backup = take(L.backup_bytes + (size_t)n_spec * 8);
    // run control: per-specimen records and stop reasons, the tile list (room
    // for the smallest tile size) and its counters
    L.run = take((size_t)n_spec * sizeof(RunSpec));
    L.done = take((size_t)n_spec * 4);
    L.tile_list = take((size_t)L.n_tiles * 4);
    L.run_count = take(4 * 4);
    // the deformation pass's own tiles (when their size differs from the
    // force pass's): halo lists, local slots, run-control list
    L.halo_a = take(((size_t)n + kTile) * k_cap * 4);
    L.halo_cnt_a = take((size_t)L.n_tiles * 4);
    L.lcol_a = take((size_t)k_cap * np * 2);
    L.tile_list_a = take((size_t)L.n_tiles * 4);
    L.total = align_up(cur);
    return L;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

}  // namespace

struct tlsph_ctx {
    Layout L;
    uint8_t* ws = nullptr;
    uint32_t flags = 0;
    DevState st{};
    std::vector<int64_t> spec_off;
    std::vector<int64_t> diag_seg_host;   // diagnostics segment table (source of an async copy)
    std::vector<DevSpec> specs;
    std::vector<DevBC> bcs;
    std::vector<RunSpec> run_host;     // staging of the run-control records
    std::vector<int32_t> done_host;
    int32_t n_bc_cap = 0;
    bool built = false;
    int parity = 0;
    int64_t nnz = 0, slots = 0;
    int64_t diag_chunks_spec = 0, diag_chunks_all = 0;
    int block_a = 256, block_b = 256, sub_b = 2;
    bool staged_ok = false;     // the staged force pass fits this device's LDS
    size_t lds_b = 0;           // its dynamic LDS bytes
    int max_lds = 0;            // LDS bytes a workgroup may use on this device
    int tile_auto = kTile;      // tile size chosen at build
    std::string last_error;
    // per-kernel timing (every timing_stride-th step while enabled)
    bool timing = false;
    int32_t timing_stride = 1;
    int64_t step_count = 0;
    int32_t contact_every = 1;     // steps between contact-list rebuilds
    int32_t contact_age = 1 << 30; // steps since the last rebuild (large: stale)
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;  // (kernel, index of start event)
    // graphs
    hipGraphExec_t gexec = nullptr;
    int graph_parity = -1;
    int graph_block_a = 0, graph_block_b = 0, graph_sub_b = 0, graph_tile = 0;
    bool graph_run = false;
    int graph_steps = 0;        // steps one replay covers (2, or twice the contact interval)
    int graph_tile_a = 0;
    bool a_own = false;         // the deformation pass runs over tiles of its own size
    int largest_b = 0;          // largest halo of the force pass's tiles
    bool run_ctl = false;       // run control set (its pointers in st while stepping)
};

namespace {

tlsph_status fail(tlsph_ctx* c, tlsph_status s, const std::string& msg) {
    if (c) c->last_error = msg;
    return s;
}

tlsph_status hip_fail(tlsph_ctx* c, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(c, TLSPH_E_HIP, m);
}

#define HIPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

template <typename T>
T* at(tlsph_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

void wire_state(tlsph_ctx* c) {
    const Layout& L = c->L;
    DevState& s = c->st;
    s.n = L.n;
    s.np = L.np;
    s.n_spec = L.n_spec;
    s.n_bc = c->n_bc_cap;
    s.flags = c->flags;
    s.XV = at<D4>(c, L.XV);
    s.spec = at<int32_t>(c, L.spec);
    s.bc = at<int32_t>(c, L.bc);
    s.perm = at<int32_t>(c, L.perm);
    s.iperm = at<int32_t>(c, L.iperm);
    s.nnb = at<int32_t>(c, L.nnb);
    s.slice_ptr = at<int64_t>(c, L.slice_ptr);
    s.col = at<int32_t>(c, L.col);
    s.col_cap = (int64_t)L.k_cap * L.np;
    s.lcol = at<uint16_t>(c, L.lcol);
    s.halo = at<int32_t>(c, L.halo);
    s.halo_cnt = at<int32_t>(c, L.halo_cnt);
    s.halo_cap = 0;
    s.tile = kTile;
    s.a_group = 1;
    s.tile_a = kTile;
    s.halo_cap_a = 0;
    s.lds_slots_a = 0;
    s.halo_a = s.halo;
    s.halo_cnt_a = s.halo_cnt;
    s.lcol_a = s.lcol;
    s.staged = 0;
    s.lds_slots = 0;
    s.Linv = at<double>(c, L.Linv);
    s.Linv32 = L.mixed ? at<float>(c, L.Linv32) : nullptr;
    s.specs = at<DevSpec>(c, L.specs);
    s.bcs = at<DevBC>(c, L.bcs);
    s.t = at<double>(c, L.t);
    s.GQ = L.mixed ? nullptr : at<GQRec<double>>(c, L.GQ);
    s.GH = L.mixed ? nullptr : at<GHRec<double>>(c, L.GH);
    s.GQ32 = L.mixed ? at<GQRec<float>>(c, L.GQ) : nullptr;
    s.GH32 = L.mixed ? at<GHRec<float>>(c, L.GH) : nullptr;
    s.U[0] = at<D4>(c, L.U0);
    s.U[1] = at<D4>(c, L.U1);
    s.VW = at<D4>(c, L.VW);
    s.sig = L.mixed ? nullptr : at<double>(c, L.sig);
    s.sig32 = L.mixed ? at<float>(c, L.sig) : nullptr;
    s.eps_p = at<double>(c, L.eps_p);
    s.eps_rate = at<double>(c, L.eps_rate);
    s.d_init = at<double>(c, L.d_init);
    s.w_p = at<double>(c, L.w_p);
    s.f_void = at<double>(c, L.f_void);
    s.e = at<double>(c, L.e);
    s.D = at<double>(c, L.D);
    s.force = at<double>(c, L.force);
    s.fvisc = at<double>(c, L.fvisc);
    s.hs = at<double>(c, L.hs);
    s.arad = at<double>(c, L.arad);
    s.ccnt = at<int32_t>(c, L.ccnt);
    s.ccol = at<int32_t>(c, L.ccol);
    s.ubuild = at<double>(c, L.ubuild);
    s.err = at<int32_t>(c, L.err);
}

DevBC to_dev(const tlsph_bc_group& g) {
    DevBC d{};
    d.mask = g.mask;
    for (int k = 0; k < 3; ++k) d.v_max[k] = g.v_max[k];
    d.tau = g.tau;
    for (int k = 0; k < 9; ++k) d.grad[k] = g.grad[k];
    return d;
}

hipEvent_t next_event(tlsph_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Contact candidate lists from the current state (positions at t^n).
tlsph_status contact_rebuild(tlsph_ctx* c, hipStream_t stream) {
    const Layout& L = c->L;
    CHash h;
    h.slot = at<CSlot>(c, L.hslot);
    h.boff = at<int32_t>(c, L.hboff);
    h.gpos = at<D4>(c, L.gpos);
    h.gref = at<D4>(c, L.gref);
    h.H = 2 * L.n_pow2;
    h.shift = 64;
    for (int64_t v = h.H; v > 1; v >>= 1) --h.shift;
    hipError_t e = launch_contact_build(c->st, c->parity, at<uint64_t>(c, L.keys),
                                        at<int32_t>(c, L.vals), h, at<double>(c, L.cbox), stream);
    if (e != hipSuccess) return hip_fail(c, e, "contact list");
    c->contact_age = 0;
    return TLSPH_OK;
}

// Run control's pointers in the kernels' state (on while it is set), and a
// fresh tile list for the current tile size.
tlsph_status run_pointers(tlsph_ctx* c, bool on, hipStream_t stream) {
    const Layout& L = c->L;
    c->st.done = on ? at<int32_t>(c, L.done) : nullptr;
    c->st.tile_list = on ? at<int32_t>(c, L.tile_list) : nullptr;
    c->st.tile_list_a = on ? at<int32_t>(c, c->a_own ? L.tile_list_a : L.tile_list) : nullptr;
    c->st.run_count = on ? at<int32_t>(c, L.run_count) : nullptr;
    if (on) {
        hipError_t e = launch_tile_list(c->st, 1, stream);
        if (e != hipSuccess) return hip_fail(c, e, "tile list");
    }
    return TLSPH_OK;
}

tlsph_status run_steps_eager(tlsph_ctx* c, int32_t n_steps, hipStream_t stream) {
    const bool mixed = c->L.mixed;
    for (int32_t k = 0; k < n_steps; ++k) {
        if (c->st.contact && c->contact_age >= c->contact_every) {
            tlsph_status cs = contact_rebuild(c, stream);
            if (cs != TLSPH_OK) return cs;
        }
        if (c->contact_age < (1 << 30)) ++c->contact_age;
        const bool timed = c->timing && (c->step_count++ % c->timing_stride) == 0;
        for (int pass = 0; pass < 2; ++pass) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) {
                const size_t idx = c->ev_used;
                e0 = next_event(c);
                e1 = next_event(c);
                if (!e0 || !e1) return fail(c, TLSPH_E_HIP, "hipEventCreate failed");
                HIPCHK(c, hipEventRecord(e0, stream));
                c->ev_marks.push_back({pass, idx});
            }
            hipError_t e = pass == 0
                               ? launch_pass_b(c->st, c->parity, c->block_b, c->sub_b, mixed,
                                               stream, c->lds_b)
                               : launch_pass_a(c->st, c->parity, c->block_a, mixed, stream);
            if (e != hipSuccess) return hip_fail(c, e, pass == 0 ? "force pass" : "deformation pass");
            if (timed) HIPCHK(c, hipEventRecord(e1, stream));
        }
        if (c->st.done) {
            hipError_t e = launch_run_control(c->st, c->parity, at<RunSpec>(c, c->L.run),
                                              at<int32_t>(c, c->L.bc_list),
                                              at<int64_t>(c, c->L.bc_ptr), stream);
            if (e == hipSuccess) e = launch_tile_list(c->st, 0, stream);
            if (e != hipSuccess) return hip_fail(c, e, "run control");
        }
        c->parity ^= 1;
    }
    return TLSPH_OK;
}

// The graph of `steps` steps from the current parity (with contact: from a
// step that rebuilds the candidate lists, `steps` twice the rebuild interval,
// so that every replay starts where the last ended).
tlsph_status ensure_graph(tlsph_ctx* c, int32_t steps, hipStream_t stream) {
    if (c->gexec && c->graph_parity == c->parity && c->graph_block_a == c->block_a &&
        c->graph_block_b == (c->st.staged ? -c->block_b : c->block_b) &&
        c->graph_sub_b == c->sub_b && c->graph_tile == c->st.tile &&
        c->graph_run == (c->st.done != nullptr) && c->graph_tile_a == c->st.tile_a &&
        c->graph_steps == steps)
        return TLSPH_OK;
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    hipGraph_t g = nullptr;
    const int p0 = c->parity;
    const int32_t age0 = c->contact_age;
    HIPCHK(c, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    const bool timing = c->timing;
    c->timing = false;
    tlsph_status s = run_steps_eager(c, steps, stream);
    c->timing = timing;
    hipError_t ce = hipStreamEndCapture(stream, &g);
    c->parity = p0;  // capture only recorded the launches
    c->contact_age = age0;
    if (s != TLSPH_OK) return s;
    if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return hip_fail(c, ie, "hipGraphInstantiate");
    c->graph_parity = p0;
    c->graph_block_a = c->block_a;
    c->graph_block_b = c->st.staged ? -c->block_b : c->block_b;
    c->graph_sub_b = c->sub_b;
    c->graph_tile = c->st.tile;
    c->graph_run = c->st.done != nullptr;
    c->graph_tile_a = c->st.tile_a;
    c->graph_steps = steps;
    return TLSPH_OK;
}

// The staged deformation pass over tiles of T particles whose largest halo
// is `largest` (lists already built): its records (56 bytes, 64 with graded
// spacing) within the default LDS limit; two tiles per workgroup where a
// tile is not a whole number of waves (one thread per particle), if both
// images fit.
void set_pass_a_shape(tlsph_ctx* c, int T, int largest) {
    const size_t la = (size_t)(T + largest) * staged_a_record_bytes(c->st.var_h != 0);
    c->st.tile_a = T;
    c->st.halo_cap_a = T * c->L.k_cap;
    c->st.lds_slots_a = T + largest;
    c->st.staged_lds_a = la <= 65536 && T + largest <= 65536 ? 1 : 0;
    c->st.a_group = (T % 64 != 0 && 2 * T <= 256 && 2 * la <= 65536) ? 2 : 1;
}

// The staged passes read halo-row entries up to kHaloPad past a tile's halo
// count without knowing the count (its rows hold n there): a force-pass
// round reads two slots per thread of at most 2 kTile threads (four lanes
// per particle stop at 128-particle tiles), a deformation-pass round four
// per thread of at most kTile.
static_assert(kHaloPad >= 2 * (2 * kTile) && kHaloPad >= 4 * kTile,
              "halo rows must be padded as far as one staging round reads");

// Halo lists and local neighbour slots for tiles of T particles into the
// given arrays; their largest halo, or -1 where the lists cannot be built
// (the sort's LDS, or staging switched off).  Synchronises.
tlsph_status build_tile_lists(tlsph_ctx* c, int T, size_t halo, size_t halo_cnt, size_t lcol,
                              int* largest, hipStream_t stream) {
    const Layout& L = c->L;
    *largest = -1;
    int E = 256;
    while (E < T * L.k_cap) E <<= 1;
    if ((2 * (size_t)E + 257) * 4 > (size_t)c->max_lds || (c->flags & TLSPH_NO_STAGING))
        return TLSPH_OK;
    const int32_t zero = 0;
    HIPCHK(c, hipMemcpyAsync(c->ws + L.err + 16, &zero, 4, hipMemcpyHostToDevice, stream));
    HIPCHK(c, launch_halo(c->st, L.k_cap, T, at<int32_t>(c, halo), at<int32_t>(c, halo_cnt),
                          at<uint16_t>(c, lcol), stream));
    int32_t lg = 0;
    HIPCHK(c, hipMemcpyAsync(&lg, c->ws + L.err + 16, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    *largest = lg;
    return TLSPH_OK;
}

// Per-tile halo lists and local neighbour slots for the force pass's tiles of
// T particles, and the LDS image size they need; the staged force pass is
// usable when the largest tile plus its halo fits one workgroup's LDS.  A
// deformation pass without tiles of its own shares them.  Synchronises.
tlsph_status set_tile_lists(tlsph_ctx* c, int T, hipStream_t stream) {
    const Layout& L = c->L;
    c->staged_ok = false;
    c->st.staged = 0;
    c->lds_b = 0;
    if (!c->a_own) {
        c->st.staged_lds_a = 0;
        c->st.a_group = 1;
        if (c->block_a == 0) c->block_a = 256;
    }
    if (T < 64 || T > kTile) return fail(c, TLSPH_E_INVALID_ARG, "tile size outside [64, 256]");
    c->st.tile = T;
    c->st.halo_cap = T * L.k_cap;
    if (!c->a_own) c->st.tile_a = T;
    int largest = -1;
    tlsph_status bs = build_tile_lists(c, T, L.halo, L.halo_cnt, L.lcol, &largest, stream);
    if (bs != TLSPH_OK || largest < 0) return bs;
    c->largest_b = largest;
    const size_t lds = (size_t)(T + largest) * staged_record_bytes(L.mixed, c->st.var_h != 0);
    if (lds <= (size_t)c->max_lds && T + largest <= 65536) {
        HIPCHK(c, prepare_staged(lds));
        c->staged_ok = true;
        c->lds_b = lds;
        c->st.lds_slots = T + largest;
        if (!c->a_own) set_pass_a_shape(c, T, largest);
    }
    return TLSPH_OK;
}

// The deformation pass's tiles: the force pass's (T equal to its tile size:
// the same arrays) or T particles of their own.  Synchronises.
tlsph_status set_tile_a_lists(tlsph_ctx* c, int T, hipStream_t stream) {
    const Layout& L = c->L;
    if (T < 64 || T > kTile) return fail(c, TLSPH_E_INVALID_ARG, "tile size outside [64, 256]");
    c->st.staged_lds_a = 0;
    c->st.a_group = 1;
    if (T == c->st.tile) {
        c->a_own = false;
        c->st.halo_a = c->st.halo;
        c->st.halo_cnt_a = c->st.halo_cnt;
        c->st.lcol_a = c->st.lcol;
        c->st.tile_a = T;
        if (c->staged_ok) set_pass_a_shape(c, T, c->largest_b);
        return TLSPH_OK;
    }
    c->a_own = true;
    c->st.halo_a = at<int32_t>(c, L.halo_a);
    c->st.halo_cnt_a = at<int32_t>(c, L.halo_cnt_a);
    c->st.lcol_a = at<uint16_t>(c, L.lcol_a);
    c->st.tile_a = T;
    int largest = -1;
    tlsph_status bs = build_tile_lists(c, T, L.halo_a, L.halo_cnt_a, L.lcol_a, &largest, stream);
    if (bs != TLSPH_OK) return bs;
    if (largest >= 0) set_pass_a_shape(c, T, largest);
    return TLSPH_OK;
}

// The same, and under run control the lists of running tiles at those sizes.
tlsph_status set_tile(tlsph_ctx* c, int T, hipStream_t stream) {
    tlsph_status ts = set_tile_lists(c, T, stream);
    if (ts == TLSPH_OK && c->st.done) ts = run_pointers(c, true, stream);
    return ts;
}

tlsph_status set_tile_a(tlsph_ctx* c, int T, hipStream_t stream) {
    tlsph_status ts = set_tile_a_lists(c, T, stream);
    if (ts == TLSPH_OK && c->st.done) ts = run_pointers(c, true, stream);
    return ts;
}

int field_comps(int f, int32_t n_spec) {
    switch (f) {
        case TLSPH_F_X: case TLSPH_F_U: case TLSPH_F_V: case TLSPH_F_FORCE: case TLSPH_F_VISC:
            return 3;
        case TLSPH_F_DEFGRAD: case TLSPH_F_Q: case TLSPH_F_LINV: case TLSPH_F_H: return 9;
        case TLSPH_F_SIGMA: return 6;
        case TLSPH_F_TIME: return -n_spec;
        case TLSPH_F_EPS_P: case TLSPH_F_EPS_P_RATE: case TLSPH_F_D_INIT: case TLSPH_F_W_P:
        case TLSPH_F_VOID: case TLSPH_F_D: case TLSPH_F_E_INT: return 1;
        default: return 0;
    }
}

}  // namespace

extern "C" {

const char* tlsph_status_string(tlsph_status s) {
    switch (s) {
        case TLSPH_OK: return "ok";
        case TLSPH_E_INVALID_ARG: return "invalid argument";
        case TLSPH_E_BAD_STATE: return "bad call order";
        case TLSPH_E_HIP: return "HIP runtime error";
        case TLSPH_E_SINGULAR_L: return "singular correction matrix";
        case TLSPH_E_NONFINITE: return "non-finite state";
        case TLSPH_E_CAPACITY: return "neighbour capacity exceeded";
        case TLSPH_E_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char* tlsph_last_error(const tlsph_ctx* c) { return c ? c->last_error.c_str() : ""; }

tlsph_status tlsph_workspace_bytes(int64_t n, int32_t n_spec, int32_t n_bc, int32_t k_cap,
                                   tlsph_precision precision, size_t* bytes) {
    if (!bytes || n < 1 || n > (int64_t)1 << 30 || n_spec < 1 || n_spec > (1 << 20) ||
        n_spec > n || n_bc < 0 || k_cap < 1 || k_cap > 512 ||
        (precision != TLSPH_FP64 && precision != TLSPH_MIXED))
        return TLSPH_E_INVALID_ARG;
    *bytes = make_layout(n, n_spec, n_bc, k_cap, precision == TLSPH_MIXED).total;
    return TLSPH_OK;
}

tlsph_status tlsph_create(int64_t n, int32_t n_spec, const int64_t* spec_offsets,
                          const tlsph_specimen* spec, int32_t n_bc, const tlsph_bc_group* bc,
                          tlsph_precision precision, int32_t k_cap, uint32_t flags,
                          void* workspace, size_t ws_bytes, hipStream_t stream, tlsph_ctx** out) {
    if (!out) return TLSPH_E_INVALID_ARG;
    *out = nullptr;
    size_t need = 0;
    if (tlsph_workspace_bytes(n, n_spec, n_bc, k_cap, precision, &need) != TLSPH_OK)
        return TLSPH_E_INVALID_ARG;
    if (!spec_offsets || !spec || (n_bc > 0 && !bc) || !workspace || ws_bytes < need ||
        ((uintptr_t)workspace % kAlign) != 0 || (flags & ~15u) != 0)
        return TLSPH_E_INVALID_ARG;
    if (spec_offsets[0] != 0 || spec_offsets[n_spec] != n) return TLSPH_E_INVALID_ARG;
    for (int32_t s = 0; s < n_spec; ++s)
        if (spec_offsets[s + 1] <= spec_offsets[s]) return TLSPH_E_INVALID_ARG;
    for (int32_t s = 0; s < n_spec; ++s) {
        const tlsph_specimen& p = spec[s];
        if (!finite_pos(p.rho0) || !finite_pos(p.E) || !finite_pos(p.c0) || !finite_pos(p.h) ||
            !finite_pos(p.dt) || !(p.nu > -1.0 && p.nu < 0.5) || p.damage < 0 || p.damage > 3 ||
            !finite_pos(p.eps_dot0) || !(p.A >= 0.0) || !(p.hg_alpha >= 0.0))
            return TLSPH_E_INVALID_ARG;
        if (p.damage == TLSPH_DMG_CL && !finite_pos(p.Wcr)) return TLSPH_E_INVALID_ARG;
        if (p.flow < TLSPH_FLOW_JC || p.flow > TLSPH_FLOW_VOCE ||
            (p.implicit_return != 0 && p.implicit_return != 1) ||
            (p.flow == TLSPH_FLOW_SWIFT && !finite_pos(p.flow_e0)) ||
            (p.flow == TLSPH_FLOW_VOCE && !(p.flow_beta >= 0.0 && p.flow_beta <= 1e300)) ||
            !(p.av_q1 >= 0.0 && p.av_q1 <= 1e300) || !(p.av_q2 >= 0.0 && p.av_q2 <= 1e300) ||
            !(p.h_per_spacing >= 0.0 && p.h_per_spacing <= 1e300) ||
            !(p.contact_k >= 0.0 && p.contact_k <= 1e300) ||
            !(p.T_star >= 0.0 && p.T_star < 1.0) || (p.T_star > 0.0 && !finite_pos(p.m)) ||
            p.newton_max_iter < 0 || p.newton_max_iter > 1000)
            return TLSPH_E_INVALID_ARG;
        if (p.damage == TLSPH_DMG_GTN &&
            (!finite_pos(p.q1) || !finite_pos(p.sN) || !(p.fF > p.fc) || !(p.fc > 0.0)))
            return TLSPH_E_INVALID_ARG;
        if (p.has_wall) {
            const double nn = p.wall_n[0] * p.wall_n[0] + p.wall_n[1] * p.wall_n[1] +
                              p.wall_n[2] * p.wall_n[2];
            if (!(fabs(nn - 1.0) < 1e-12)) return TLSPH_E_INVALID_ARG;
        }
    }
    for (int32_t g = 0; g < n_bc; ++g)
        if (bc[g].mask < 0 || bc[g].mask > 7 || !(bc[g].tau >= 0.0)) return TLSPH_E_INVALID_ARG;

    tlsph_ctx* c = new tlsph_ctx();
    c->L = make_layout(n, n_spec, n_bc, k_cap, precision == TLSPH_MIXED);
    c->ws = static_cast<uint8_t*>(workspace);
    c->flags = flags;
    c->n_bc_cap = n_bc;
    c->spec_off.assign(spec_offsets, spec_offsets + n_spec + 1);
    c->specs.resize(n_spec);
    for (int32_t s = 0; s < n_spec; ++s) {
        const tlsph_specimen& p = spec[s];
        DevSpec& d = c->specs[s];
        d.rho0 = p.rho0; d.E = p.E; d.nu = p.nu; d.c0 = p.c0; d.S_alpha = p.S_alpha;
        // a constant homologous temperature multiplies every flow law by
        // 1 - T*^m (eq. JC_viscoplastic_model) and the Johnson-Cook failure
        // strain by 1 + D5 T* (Sec. 5.2): both are folded into the constants
        const double theta = p.T_star > 0.0 ? 1.0 - pow(p.T_star, p.m) : 1.0;
        const double tf = 1.0 + p.D5 * p.T_star;
        d.Gamma0 = p.Gamma0; d.A = p.A * theta; d.B = p.B * theta; d.n = p.n; d.C = p.C;
        d.eps_dot0 = p.eps_dot0;
        d.Wcr = p.Wcr; d.D1 = p.D1 * tf; d.D2 = p.D2 * tf; d.D3 = p.D3; d.D4 = p.D4; d.D5 = p.D5;
        d.q1 = p.q1; d.q2 = p.q2; d.q3 = p.q3; d.f0 = p.f0; d.fN = p.fN; d.eN = p.eN;
        d.sN = p.sN; d.fc = p.fc; d.fF = p.fF; d.k_omega = p.k_omega;
        d.h = p.h; d.dt = p.dt; d.hg_alpha = p.hg_alpha;
        for (int k = 0; k < 3; ++k) d.wall_n[k] = p.wall_n[k];
        d.wall_d = p.wall_d;
        d.G = p.E / (2.0 * (1.0 + p.nu));
        d.inv_h = 1.0 / p.h;
        d.wnorm = 8.0 / (M_PI * p.h * p.h * p.h);
        d.h2 = p.h * p.h;
        d.inv_cell = 1.0 / (p.h * (1.0 + 1e-9));
        d.inv_dt = 1.0 / p.dt;
        d.inv_rho0 = 1.0 / p.rho0;
        d.inv_eps_dot0 = 1.0 / p.eps_dot0;
        d.grad_k = d.wnorm * d.inv_h;
        d.hg_k = -p.hg_alpha * p.E * d.wnorm;
        d.dt_rho0 = p.dt / p.rho0;
        d.damage = p.damage;
        d.has_wall = p.has_wall;
        d.flow = p.flow;
        d.implicit_return = p.implicit_return;
        d.flow_e0 = p.flow_e0;
        d.flow_beta = p.flow_beta;
        d.av_q1 = p.av_q1;
        d.av_q2 = p.av_q2;
        d.h_per_spacing = p.h_per_spacing;
        d.contact_k = p.contact_k;
        d.contact_comp = (1.0 - p.nu * p.nu) / p.E;
        d.newton_gtn = p.newton_max_iter > 0 ? p.newton_max_iter : 50;
        d.newton_impl = p.newton_max_iter > 0 ? p.newton_max_iter : 100;
        d.first = spec_offsets[s];
        d.last = spec_offsets[s + 1];
    }
    c->bcs.resize(n_bc > 0 ? n_bc : 1);
    for (int32_t g = 0; g < n_bc; ++g) c->bcs[g] = to_dev(bc[g]);
    wire_state(c);
    // the deformation pass is compiled per damage model (or for any) and
    // with Johnson-Cook hardening and the explicit return only (or any law)
    c->st.model = spec[0].damage;
    c->st.flow_general = 0;
    c->st.av = 0;
    c->st.var_h = 0;
    c->st.contact = 0;
    c->st.contact_skin = 0.0;
    for (int32_t q = 0; q < n_spec; ++q) {
        if (spec[q].h_per_spacing > 0.0) c->st.var_h = 1;
        if (spec[q].contact_k > 0.0) c->st.contact = 1;
        if (spec[q].damage != spec[0].damage) c->st.model = -1;
        if (spec[q].av_q1 != 0.0 || spec[q].av_q2 != 0.0) c->st.av = 1;
        if (spec[q].flow != TLSPH_FLOW_JC || spec[q].implicit_return != 0 || c->st.av)
            c->st.flow_general = 1;
    }

    const Layout& L = c->L;
    hipError_t e = hipMemcpyAsync(c->ws + L.specs, c->specs.data(), n_spec * sizeof(DevSpec),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && n_bc > 0)
        e = hipMemcpyAsync(c->ws + L.bcs, c->bcs.data(), n_bc * sizeof(DevBC),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + L.spec_off, c->spec_off.data(), (n_spec + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        delete c;
        return TLSPH_E_HIP;
    }
    *out = c;
    return TLSPH_OK;
}

tlsph_status tlsph_build_neighbors(tlsph_ctx* c, const double* X, const double* V0,
                                   const int32_t* bc_group, hipStream_t stream) {
    if (!c || !X || !V0 || !bc_group) return fail(c, TLSPH_E_INVALID_ARG, "null argument");
    const Layout& L = c->L;
    c->built = false;
    c->parity = 0;
    c->run_ctl = false;
    c->st.done = c->st.tile_list = c->st.run_count = nullptr;
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    // error words: first singular = INT_MAX, max count = 0, flags = 0, build = 0
    const int32_t init_err[8] = {0x7fffffff, 0, 0, 0, 0, 0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(c->ws + L.err, init_err, sizeof init_err, hipMemcpyHostToDevice, stream));
    BuildBuffers b{};
    b.X_in = X;
    b.V0_in = V0;
    b.bc_in = bc_group;
    b.spec_off = at<int64_t>(c, L.spec_off);
    b.bbox = at<double>(c, L.bbox);
    b.keys = at<uint64_t>(c, L.keys);
    b.vals = at<int32_t>(c, L.vals);
    b.n_pow2 = L.n_pow2;
    HIPCHK(c, launch_build_count(c->st, b, stream));
    int32_t err[8];
    int64_t total_slots = 0;
    HIPCHK(c, hipMemcpyAsync(err, c->ws + L.err, sizeof err, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipMemcpyAsync(&total_slots, c->ws + L.slice_ptr + L.n_slices * 8, 8,
                             hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    if (err[3] & 2) return fail(c, TLSPH_E_INVALID_ARG, "bc_group entry outside [-1, n_bc)");
    if (err[3] & 1) return fail(c, TLSPH_E_UNSUPPORTED, "more than 16384 cells along an axis");
    if (err[1] > L.k_cap || total_slots > (int64_t)L.k_cap * L.np)
        return fail(c, TLSPH_E_CAPACITY, "a particle has " + std::to_string(err[1]) +
                                             " neighbours, k_cap is " + std::to_string(L.k_cap));
    HIPCHK(c, launch_build_fill(c->st, b, stream));
    c->st.staged = 0;
    c->staged_ok = false;
    c->a_own = false;
    c->st.halo_a = c->st.halo;
    c->st.halo_cnt_a = c->st.halo_cnt;
    c->st.lcol_a = c->st.lcol;
    c->lds_b = 0;
    c->block_b = 256;
    c->sub_b = 2;
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&c->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // Tile size of the staged force pass: whole rounds of tiles over the
    // compute units (one tile per CU at a time), at most kTile particles.
    int n_cu = 0;
    HIPCHK(c, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (n_cu < 1) n_cu = 1;
    {
        const int64_t per_round = (int64_t)kTile * n_cu;
        const int64_t rounds = (L.n + per_round - 1) / per_round;
        int64_t T = (L.n + rounds * n_cu - 1) / (rounds * n_cu);
        c->tile_auto = (int)(T < 64 ? 64 : (T > kTile ? kTile : T));
    }
    HIPCHK(c, launch_shape_and_init(c->st, L.mixed, stream));
    HIPCHK(c, launch_bc_lists(c->st, b.keys, b.vals, L.n_pow2, at<int32_t>(c, L.bc_list),
                              at<int64_t>(c, L.bc_ptr), stream));
    HIPCHK(c, hipMemcpyAsync(err, c->ws + L.err, sizeof err, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    if (err[0] != 0x7fffffff) {
        int32_t orig = -1;
        HIPCHK(c, hipMemcpyAsync(&orig, c->ws + L.perm + (size_t)err[0] * 4, 4,
                                 hipMemcpyDeviceToHost, stream));
        HIPCHK(c, hipStreamSynchronize(stream));
        return fail(c, TLSPH_E_SINGULAR_L,
                    "singular correction matrix at particle " + std::to_string(orig));
    }
    // LDS staging of the force pass: per-tile halo lists when they fit
    {
        tlsph_status ts = set_tile(c, c->tile_auto, stream);
        if (ts != TLSPH_OK) return ts;
        if (c->staged_ok) {
            c->st.staged = 1;
            c->block_b = c->st.tile * c->sub_b;
        }
    }
    // group sizes and neighbour counts to the host (one synchronisation)
    std::vector<int64_t> bptr((size_t)L.n_bc + 1, 0);
    std::vector<int32_t> cnt(L.np);
    if (L.n_bc > 0)
        HIPCHK(c, hipMemcpyAsync(bptr.data(), c->ws + L.bc_ptr, bptr.size() * 8,
                                 hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipMemcpyAsync(cnt.data(), c->ws + L.nnb, L.np * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    // diagnostics segments: chunks of each specimen, then of each group
    {
        std::vector<int64_t>& seg = c->diag_seg_host;
        seg.assign((size_t)L.n_spec + L.n_bc + 1, 0);
        auto chunks = [](int64_t m) { return m > 0 ? (m + kDiagChunk - 1) / kDiagChunk : 1; };
        for (int32_t q = 0; q < L.n_spec; ++q)
            seg[q + 1] = seg[q] + chunks(c->spec_off[q + 1] - c->spec_off[q]);
        for (int32_t g = 0; g < L.n_bc; ++g)
            seg[L.n_spec + g + 1] = seg[L.n_spec + g] + chunks(bptr[g + 1] - bptr[g]);
        if (seg.back() > L.diag_chunk_cap)
            return fail(c, TLSPH_E_HIP, "diagnostics chunk table exceeds its capacity");
        // (the host table lives in the context, so the copy may complete later)
        HIPCHK(c, hipMemcpyAsync(c->ws + L.diag_seg, seg.data(), seg.size() * 8,
                                 hipMemcpyHostToDevice, stream));
        c->diag_chunks_spec = seg[L.n_spec];
        c->diag_chunks_all = seg.back();
    }
    // neighbour pairs: sum of counts
    int64_t nnz = 0;
    for (int64_t p = 0; p < L.n; ++p) nnz += cnt[p];
    c->nnz = nnz;
    c->slots = total_slots;
    c->built = true;
    if (c->st.contact) {   // a valid list before any force pass (autotune included)
        tlsph_status cs = contact_rebuild(c, stream);
        if (cs != TLSPH_OK) return cs;
        c->contact_age = 1 << 30;
    }
    return TLSPH_OK;
}

tlsph_status tlsph_step(tlsph_ctx* c, int32_t n_steps, hipStream_t stream) {
    if (!c) return TLSPH_E_INVALID_ARG;
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "step before build");
    if (n_steps < 0) return fail(c, TLSPH_E_INVALID_ARG, "negative step count");
    bool graphs = (c->flags & TLSPH_USE_GRAPHS) && !c->timing && n_steps >= 2 &&
                  stream != nullptr;
    if (graphs) {
        // a caller that is capturing already records the plain launches
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIPCHK(c, hipStreamIsCapturing(stream, &cs));
        graphs = cs == hipStreamCaptureStatusNone;
    }
    if (!graphs) return run_steps_eager(c, n_steps, stream);
    int32_t left = n_steps;
    if (c->st.contact) {
        // replays of twice the rebuild interval, each from a step that
        // rebuilds the lists: eager steps up to the next such step, and on
        // to the one after if the parity differs from the graph's
        const int32_t every = c->contact_every;
        const int32_t G = 2 * every;
        auto eager_to_rebuild = [&]() -> tlsph_status {
            while (left > 0 && c->contact_age < every) {
                tlsph_status s = run_steps_eager(c, 1, stream);
                if (s != TLSPH_OK) return s;
                --left;
            }
            return TLSPH_OK;
        };
        tlsph_status s = eager_to_rebuild();
        if (s != TLSPH_OK) return s;
        if (c->gexec && c->graph_steps == G && c->graph_parity != c->parity && left >= every + G) {
            s = run_steps_eager(c, every, stream);
            if (s != TLSPH_OK) return s;
            left -= every;
        }
        if (left >= G) {
            s = ensure_graph(c, G, stream);
            if (s != TLSPH_OK) return s;
            for (; left >= G; left -= G) HIPCHK(c, hipGraphLaunch(c->gexec, stream));
            c->contact_age = every;   // each replay ends where the next rebuild is due
        }
        if (left) return run_steps_eager(c, left, stream);
        return TLSPH_OK;
    }
    if (c->gexec && c->graph_parity != c->parity) {
        tlsph_status s = run_steps_eager(c, 1, stream);
        if (s != TLSPH_OK) return s;
        --left;
    }
    if (left >= 2) {
        tlsph_status s = ensure_graph(c, 2, stream);
        if (s != TLSPH_OK) return s;
        for (; left >= 2; left -= 2) HIPCHK(c, hipGraphLaunch(c->gexec, stream));
    }
    if (left) return run_steps_eager(c, left, stream);
    return TLSPH_OK;
}

tlsph_status tlsph_get_state(tlsph_ctx* c, tlsph_field field, double* dst, size_t bytes,
                             hipStream_t stream) {
    if (!c) return TLSPH_E_INVALID_ARG;
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "get_state before build");
    const int comps = field_comps(field, c->L.n_spec);
    if (!dst || comps == 0) return fail(c, TLSPH_E_INVALID_ARG, "bad field or null dst");
    const size_t need = comps > 0 ? (size_t)comps * c->L.n * 8 : (size_t)(-comps) * 8;
    if (bytes != need) return fail(c, TLSPH_E_INVALID_ARG, "wrong byte count");
    if (field == TLSPH_F_TIME) {
        HIPCHK(c, hipMemcpyAsync(dst, c->st.t, need, hipMemcpyDeviceToDevice, stream));
        return TLSPH_OK;
    }
    HIPCHK(c, launch_get_field(c->st, field, c->parity, c->L.mixed, dst, stream));
    return TLSPH_OK;
}

tlsph_status tlsph_set_state(tlsph_ctx* c, tlsph_field field, const double* src, size_t bytes,
                             hipStream_t stream) {
    if (!c) return TLSPH_E_INVALID_ARG;
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "set_state before build");
    const int comps = field_comps(field, c->L.n_spec);
    if (!src || comps == 0 || field == TLSPH_F_X || field == TLSPH_F_FORCE ||
        field == TLSPH_F_LINV)
        return fail(c, TLSPH_E_INVALID_ARG, "bad or read-only field, or null src");
    const size_t need = comps > 0 ? (size_t)comps * c->L.n * 8 : (size_t)(-comps) * 8;
    if (bytes != need) return fail(c, TLSPH_E_INVALID_ARG, "wrong byte count");
    if (field == TLSPH_F_TIME) {
        HIPCHK(c, hipMemcpyAsync(c->st.t, src, need, hipMemcpyDeviceToDevice, stream));
        return TLSPH_OK;
    }
    HIPCHK(c, launch_set_field(c->st, field, c->parity, c->L.mixed, src, stream));
    c->contact_age = 1 << 30;   // positions may have changed
    return TLSPH_OK;
}

tlsph_status tlsph_set_contact(tlsph_ctx* c, int32_t every, double skin) {
    if (!c) return TLSPH_E_INVALID_ARG;
    if (every < 1 || !(skin >= 0.0 && skin <= 1e300))
        return fail(c, TLSPH_E_INVALID_ARG, "contact: every >= 1 and a finite skin >= 0");
    c->contact_every = every;
    c->st.contact_skin = skin;
    c->contact_age = 1 << 30;
    return TLSPH_OK;
}

tlsph_status tlsph_set_run_control(tlsph_ctx* c, const tlsph_stop_rule* rules,
                                   hipStream_t stream) {
    if (!c) return TLSPH_E_INVALID_ARG;
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "run control before build");
    const Layout& L = c->L;
    if (!rules) {
        c->run_ctl = false;
        tlsph_status r = run_pointers(c, false, stream);
        if (r != TLSPH_OK) return r;
        HIPCHK(c, hipStreamSynchronize(stream));
        return TLSPH_OK;
    }
    for (int32_t q = 0; q < L.n_spec; ++q) {
        const tlsph_stop_rule& r = rules[q];
        if (r.step_cap < 0 || r.group < -1 || r.group >= c->n_bc_cap || r.axis < 0 ||
            r.axis > 2 || !(r.sign == 1.0 || r.sign == -1.0) || !(r.drop > 0.0 && r.drop < 1.0) ||
            !(r.min_peak >= 0.0 && r.min_peak <= 1e300))
            return fail(c, TLSPH_E_INVALID_ARG, "stop rule of specimen " + std::to_string(q));
    }
    c->run_host.assign(L.n_spec, RunSpec{});
    c->done_host.assign(L.n_spec, kRunning);
    for (int32_t q = 0; q < L.n_spec; ++q) {
        RunSpec& d = c->run_host[q];
        d.cap = rules[q].step_cap;
        d.steps = 0;
        d.sign = rules[q].sign;
        d.drop = rules[q].drop;
        d.min_peak = rules[q].min_peak;
        d.peak = 0.0;
        d.last = 0.0;
        d.group = rules[q].group;
        d.axis = rules[q].axis;
    }
    HIPCHK(c, hipMemcpyAsync(c->ws + L.run, c->run_host.data(), L.n_spec * sizeof(RunSpec),
                             hipMemcpyHostToDevice, stream));
    HIPCHK(c, hipMemcpyAsync(c->ws + L.done, c->done_host.data(), L.n_spec * 4,
                             hipMemcpyHostToDevice, stream));
    c->run_ctl = true;
    tlsph_status r = run_pointers(c, true, stream);
    if (r != TLSPH_OK) return r;
    HIPCHK(c, hipStreamSynchronize(stream));
    return TLSPH_OK;
}

tlsph_status tlsph_get_run_status(tlsph_ctx* c, int32_t* why, int64_t* steps, double* peak,
                                  int32_t* n_running, hipStream_t stream) {
    if (!c) return TLSPH_E_INVALID_ARG;
    if (!c->run_ctl) return fail(c, TLSPH_E_BAD_STATE, "no run control set");
    const Layout& L = c->L;
    int32_t cnt[4] = {0, 0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(c->run_host.data(), c->ws + L.run, L.n_spec * sizeof(RunSpec),
                             hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipMemcpyAsync(c->done_host.data(), c->ws + L.done, L.n_spec * 4,
                             hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipMemcpyAsync(cnt, c->ws + L.run_count, sizeof cnt, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    for (int32_t q = 0; q < L.n_spec; ++q) {
        if (why) why[q] = c->done_host[q];
        if (steps) steps[q] = c->run_host[q].steps;
        if (peak) peak[q] = c->run_host[q].peak;
    }
    if (n_running) *n_running = cnt[2];
    return TLSPH_OK;
}

tlsph_status tlsph_run(tlsph_ctx* c, int64_t max_steps, int32_t check_every, int64_t* steps_run,
                       hipStream_t stream) {
    if (!c) return TLSPH_E_INVALID_ARG;
    if (steps_run) *steps_run = 0;
    if (!c->run_ctl) return fail(c, TLSPH_E_BAD_STATE, "no run control set");
    if (max_steps < 0 || check_every < 1)
        return fail(c, TLSPH_E_INVALID_ARG, "max_steps >= 0 and check_every >= 1");
    int64_t done = 0;
    int32_t running = 0;
    HIPCHK(c, hipMemcpyAsync(&running, c->ws + c->L.run_count + 8, 4, hipMemcpyDeviceToHost,
                             stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    while (done < max_steps && running > 0) {
        const int32_t k = (int32_t)std::min<int64_t>(check_every, max_steps - done);
        tlsph_status r = tlsph_step(c, k, stream);
        if (r != TLSPH_OK) return r;
        done += k;
        if (steps_run) *steps_run = done;
        HIPCHK(c, hipMemcpyAsync(&running, c->ws + c->L.run_count + 8, 4, hipMemcpyDeviceToHost,
                                 stream));
        HIPCHK(c, hipStreamSynchronize(stream));
    }
    return TLSPH_OK;
}

tlsph_status tlsph_neighbor_count(const tlsph_ctx* c, int64_t* nnz) {
    if (!c || !nnz) return TLSPH_E_INVALID_ARG;
    if (!c->built) return TLSPH_E_BAD_STATE;
    *nnz = c->nnz;
    return TLSPH_OK;
}

tlsph_status tlsph_get_neighbors(tlsph_ctx* c, int64_t* row_ptr, int32_t* col, hipStream_t stream) {
    if (!c || !row_ptr || !col) return fail(c, TLSPH_E_INVALID_ARG, "null argument");
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "get_neighbors before build");
    HIPCHK(c, launch_export_neighbors(c->st, row_ptr, col, nullptr, stream));
    return TLSPH_OK;
}

tlsph_status tlsph_get_diagnostics(tlsph_ctx* c, double* spec_diag, double* bc_diag,
                                   hipStream_t stream) {
    if (!c || !spec_diag) return fail(c, TLSPH_E_INVALID_ARG, "null argument");
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "diagnostics before build");
    const bool groups = bc_diag != nullptr && c->L.n_bc > 0;
    HIPCHK(c, launch_diagnostics(c->st, c->parity, at<int32_t>(c, c->L.bc_list),
                                 at<int64_t>(c, c->L.bc_ptr), at<int64_t>(c, c->L.diag_seg),
                                 groups ? c->L.n_spec + c->L.n_bc : c->L.n_spec,
                                 groups ? c->diag_chunks_all : c->diag_chunks_spec,
                                 at<double>(c, c->L.diag_part), spec_diag, bc_diag, stream));
    return TLSPH_OK;
}

tlsph_status tlsph_get_diagnostics_static(tlsph_ctx* c, double* spec_diag, double* bc_diag,
                                          hipStream_t stream) {
    if (!c || !spec_diag) return fail(c, TLSPH_E_INVALID_ARG, "null argument");
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "diagnostics before build");
    const bool groups = bc_diag != nullptr && c->L.n_bc > 0;
    const int64_t chunks = groups ? c->diag_chunks_all : c->diag_chunks_spec;
    if (chunks * kNDiag > kScratchDoubles)
        return fail(c, TLSPH_E_CAPACITY,
                    "diagnostics need " + std::to_string(chunks) + " chunk partials; the static "
                    "scratch holds " + std::to_string(kScratchDoubles / kNDiag) +
                    " (use tlsph_get_diagnostics)");
    double* part = nullptr;
    HIPCHK(c, scratch_ptr(&part));
    HIPCHK(c, launch_diagnostics(c->st, c->parity, at<int32_t>(c, c->L.bc_list),
                                 at<int64_t>(c, c->L.bc_ptr), at<int64_t>(c, c->L.diag_seg),
                                 groups ? c->L.n_spec + c->L.n_bc : c->L.n_spec, chunks, part,
                                 spec_diag, bc_diag, stream));
    return TLSPH_OK;
}

tlsph_status tlsph_set_bc_groups(tlsph_ctx* c, int32_t n_bc, const tlsph_bc_group* bc,
                                 hipStream_t stream) {
    if (!c || n_bc < 0 || n_bc > c->n_bc_cap || (n_bc > 0 && !bc))
        return fail(c, TLSPH_E_INVALID_ARG, "bad group table");
    for (int32_t g = 0; g < n_bc; ++g) {
        if (bc[g].mask < 0 || bc[g].mask > 7 || !(bc[g].tau >= 0.0))
            return fail(c, TLSPH_E_INVALID_ARG, "bad group");
        c->bcs[g] = to_dev(bc[g]);
    }
    if (n_bc > 0)
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.bcs, c->bcs.data(), n_bc * sizeof(DevBC),
                                 hipMemcpyHostToDevice, stream));
    return TLSPH_OK;
}

tlsph_status tlsph_enable_kernel_timing(tlsph_ctx* c, int32_t stride) {
    if (!c || stride < 0) return TLSPH_E_INVALID_ARG;
    c->timing = stride > 0;
    c->timing_stride = stride > 0 ? stride : 1;
    c->step_count = 0;
    return TLSPH_OK;
}

tlsph_status tlsph_kernel_times(tlsph_ctx* c, double ms[2], int64_t launches[2]) {
    if (!c || !ms || !launches) return TLSPH_E_INVALID_ARG;
    ms[0] = ms[1] = 0.0;
    launches[0] = launches[1] = 0;
    if (c->ev_used > 0) HIPCHK(c, hipEventSynchronize(c->ev_pool[c->ev_used - 1]));
    for (auto& m : c->ev_marks) {
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev_pool[m.second], c->ev_pool[m.second + 1]));
        ms[m.first] += t;
        launches[m.first] += 1;
    }
    c->ev_marks.clear();
    c->ev_used = 0;
    return TLSPH_OK;
}

static tlsph_status autotune_all(tlsph_ctx* c, hipStream_t stream) {
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "autotune before build");
    const Layout& L = c->L;
    uint8_t* state = c->ws + L.state_begin;
    uint8_t* backup = c->ws + L.backup;
    HIPCHK(c, hipMemcpyAsync(backup, state, L.backup_bytes, hipMemcpyDeviceToDevice, stream));
    HIPCHK(c, hipMemcpyAsync(backup + L.backup_bytes, c->st.t, L.n_spec * 8,
                             hipMemcpyDeviceToDevice, stream));
    // the sticky error flags too: the timing runs repeat single passes on
    // states no step would produce, which may raise flags of their own
    int32_t flags_before = 0;
    HIPCHK(c, hipMemcpyAsync(&flags_before, c->ws + L.err + 8, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    // force pass: unstaged (lanes per particle, block) and staged (tile
    // size, lanes per particle); deformation pass: block
    struct Cand { int staged, sub, block, tile; };
    const Cand cand_u[] = {{0, 4, 256, 0}, {0, 4, 128, 0}, {0, 2, 128, 0}, {0, 1, 64, 0},
                           {0, 1, 128, 0}, {0, 1, 256, 0}};
    const int cand_a[] = {64, 128, 256};   // (staged: per tile size below)
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    const int reps = 10;   // launches timed per candidate (their spread is about 2 %)
    auto timed = [&](auto&& launch, float* ms) -> tlsph_status {
        // every candidate starts from the saved state
        HIPCHK(c, hipMemcpyAsync(state, backup, L.backup_bytes, hipMemcpyDeviceToDevice, stream));
        hipError_t e = hipSuccess;
        for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
            if (r == 1) HIPCHK(c, hipEventRecord(e0, stream));
            e = launch();
        }
        if (e != hipSuccess) return hip_fail(c, e, "autotune launch");
        HIPCHK(c, hipEventRecord(e1, stream));
        HIPCHK(c, hipEventSynchronize(e1));
        HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
        return TLSPH_OK;
    };
    // The two passes are timed separately: unstaged candidates do not depend
    // on the tile size, staged ones are timed per tile size.
    auto time_b = [&](int staged, int sub, int block, float* ms) -> tlsph_status {
        c->st.staged = staged;
        const int blk = staged ? c->st.tile * sub : block;
        return timed([&] {
            return launch_pass_b(c->st, c->parity, blk, sub, L.mixed, stream, c->lds_b);
        }, ms);
    };
    auto time_a = [&](int block, float* ms) -> tlsph_status {
        return timed([&] { return launch_pass_a(c->st, c->parity, block, L.mixed, stream); }, ms);
    };
    // Each pass's fastest shape, chosen on its own: the force pass unstaged
    // (lanes, block) or staged (tile size, lanes); the deformation pass
    // unstaged (block) or staged over tiles of some size, its own or the
    // force pass's.  Candidates for the deformation pass's tiles are timed
    // on the force pass's lists of that size.
    c->a_own = false;
    c->st.halo_a = c->st.halo;
    c->st.halo_cnt_a = c->st.halo_cnt;
    c->st.lcol_a = c->st.lcol;
    float bu = 1e30f, au = 1e30f;
    int bu_sub = 2, bu_blk = 256, au_blk = 256;
    for (const Cand& k : cand_u) {
        float t = 0.0f;
        tlsph_status st = time_b(0, k.sub, k.block, &t);
        if (st != TLSPH_OK) return st;
        if (t < bu) { bu = t; bu_sub = k.sub; bu_blk = k.block; }
    }
    for (int blk : cand_a) {
        float t = 0.0f;
        tlsph_status st = time_a(blk, &t);
        if (st != TLSPH_OK) return st;
        if (t < au) { au = t; au_blk = blk; }
    }
    float bs_best = 1e30f, as_best = 1e30f;
    int bs_sub = 2, bs_tile = 0, as_tile = 0;
    if (!(c->flags & TLSPH_NO_STAGING)) {
        // Tile sizes: the build's, six fixed ones, and for each of those
        // the sizes that fill whole rounds at the number of workgroups per
        // CU the force pass's LDS image allows (the next smaller, and a few
        // percent larger if that drops a barely started last round).
        int dev = 0, lds_cu = 0, n_cu = 0;
        HIPCHK(c, hipGetDevice(&dev));
        HIPCHK(c, hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                        dev));
        HIPCHK(c, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        if (lds_cu < c->max_lds) lds_cu = c->max_lds;
        if (n_cu < 1) n_cu = 1;
        std::vector<int> tiles = {c->tile_auto, 128, 112, 96, 88, 80, 64};
        const size_t n_fixed = tiles.size();
        for (size_t q = 0; q < tiles.size(); ++q) {
            bool seen = false;
            for (size_t r = 0; r < q; ++r) seen = seen || tiles[r] == tiles[q];
            if (seen) continue;
            tlsph_status ts = set_tile(c, tiles[q], stream);
            if (ts != TLSPH_OK) return ts;
            if (!c->staged_ok) continue;
            for (int sub : {4, 2, 1}) {
                if (tiles[q] > staged_tile_max(sub)) continue;
                float t = 0.0f;
                tlsph_status st = time_b(1, sub, 0, &t);
                if (st != TLSPH_OK) return st;
                if (t < bs_best) { bs_best = t; bs_sub = sub; bs_tile = tiles[q]; }
            }
            if (c->st.staged_lds_a) {
                float t = 0.0f;
                tlsph_status st = time_a(0, &t);
                if (st != TLSPH_OK) return st;
                if (t < as_best) { as_best = t; as_tile = tiles[q]; }
            }
            const int64_t w = (int64_t)lds_cu / (int64_t)c->lds_b;
            if (w >= 1 && q < n_fixed) {
                const int64_t slots = w * n_cu;
                const int64_t rounds = (L.n + (int64_t)tiles[q] * slots - 1) /
                                       ((int64_t)tiles[q] * slots);
                const int64_t T1 = (L.n + rounds * slots - 1) / (rounds * slots);
                if (T1 >= 64 && T1 < tiles[q]) tiles.push_back((int)T1);
                const int64_t full = L.n / ((int64_t)tiles[q] * slots);
                if (full >= 1) {
                    const int64_t T2 = (L.n + full * slots - 1) / (full * slots);
                    if (T2 > tiles[q] && T2 <= kTile && T2 * 100 <= (int64_t)tiles[q] * 108)
                        tiles.push_back((int)T2);
                }
            }
        }
    }
    // apply: the force pass's tiles (or, unstaged, the deformation pass's
    // staged size, or the build's), then the deformation pass's
    {
        const bool b_staged = bs_best < bu;
        const bool a_staged = as_best < au;
        const int tb = b_staged ? bs_tile : (a_staged ? as_tile : c->tile_auto);
        tlsph_status ts = set_tile(c, tb, stream);
        if (ts != TLSPH_OK) return ts;
        const bool ok_b = !b_staged || c->staged_ok;
        c->st.staged = b_staged && ok_b;
        c->sub_b = b_staged && ok_b ? bs_sub : bu_sub;
        c->block_b = c->st.staged ? c->st.tile * c->sub_b : bu_blk;
        c->block_a = au_blk;
        if (a_staged) {
            ts = set_tile_a(c, as_tile, stream);
            if (ts != TLSPH_OK) return ts;
            if (c->st.staged_lds_a) c->block_a = 0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(c, hipMemcpyAsync(state, backup, L.backup_bytes, hipMemcpyDeviceToDevice, stream));
    HIPCHK(c, hipMemcpyAsync(c->st.t, backup + L.backup_bytes, L.n_spec * 8,
                             hipMemcpyDeviceToDevice, stream));
    HIPCHK(c, hipMemcpyAsync(c->ws + L.err + 8, &flags_before, 4, hipMemcpyHostToDevice, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    c->contact_age = 1 << 30;
    return TLSPH_OK;
}

tlsph_status tlsph_autotune(tlsph_ctx* c, hipStream_t stream) {
    if (!c) return TLSPH_E_INVALID_ARG;
    // the candidates are timed over every specimen, with run control
    // suspended (the state is restored afterwards)
    const bool rc = c->st.done != nullptr;
    if (rc) {
        tlsph_status r = run_pointers(c, false, stream);
        if (r != TLSPH_OK) return r;
    }
    tlsph_status s = autotune_all(c, stream);
    if (rc) {
        tlsph_status r = run_pointers(c, true, stream);
        if (s == TLSPH_OK) s = r;
    }
    return s;
}

tlsph_status tlsph_info(tlsph_ctx* c, int64_t out[9], hipStream_t stream) {
    if (!c || !out) return TLSPH_E_INVALID_ARG;
    out[0] = c->st.staged ? -c->block_b : c->block_b;
    out[1] = c->block_a == 0 && c->a_own ? -c->st.tile_a : c->block_a;
    out[2] = c->nnz;
    out[3] = c->slots;
    out[4] = c->L.n;
    out[5] = 0;
    out[6] = c->sub_b;
    out[7] = c->st.staged ? (int64_t)c->lds_b : 0;
    out[8] = c->st.staged ? c->st.tile : 0;
    if (c->built) {
        int32_t fl = 0;
        HIPCHK(c, hipMemcpyAsync(&fl, c->ws + c->L.err + 8, 4, hipMemcpyDeviceToHost, stream));
        HIPCHK(c, hipStreamSynchronize(stream));
        out[5] = fl;
    }
    return TLSPH_OK;
}

tlsph_status tlsph_set_launch_shape(tlsph_ctx* c, const int32_t shape[5], hipStream_t stream) {
    if (!c || !shape) return TLSPH_E_INVALID_ARG;
    if (!c->built) return fail(c, TLSPH_E_BAD_STATE, "launch shape before build");
    const int32_t staged = shape[0], sub = shape[1], blk_b = shape[2], blk_a = shape[3];
    const int32_t tile = shape[4] == 0 ? c->tile_auto : shape[4];
    if (staged != 0 && staged != 1) return fail(c, TLSPH_E_INVALID_ARG, "staged must be 0 or 1");
    if (sub != 1 && sub != 2 && sub != 4) return fail(c, TLSPH_E_INVALID_ARG, "lanes per particle");
    if (!staged && (blk_b < 64 || blk_b > 256 || blk_b % 64 != 0))
        return fail(c, TLSPH_E_INVALID_ARG, "force-pass block must be 64, 128, 192 or 256");
    if (blk_a > 0 && (blk_a < 64 || blk_a > 256 || blk_a % 64 != 0))
        return fail(c, TLSPH_E_INVALID_ARG,
                    "deformation-pass block must be 64, 128, 192 or 256, 0 (staged over the "
                    "force pass's tiles) or -T (staged over tiles of its own, T in [64, 256])");
    if (blk_a < 0 && (-blk_a < 64 || -blk_a > kTile))
        return fail(c, TLSPH_E_INVALID_ARG, "the deformation pass's tiles hold 64 to 256 particles");
    if ((staged || blk_a == 0) && (tile < 64 || tile > kTile))
        return fail(c, TLSPH_E_INVALID_ARG, "tile must hold 64 to 256 particles");
    if (staged && tile > staged_tile_max(sub))
        return fail(c, TLSPH_E_UNSUPPORTED, "four lanes per particle run tiles of at most 128");
    if ((staged || blk_a == 0) && (tile != c->st.tile || !c->staged_ok)) {
        tlsph_status ts = set_tile(c, tile, stream);
        if (ts != TLSPH_OK) return ts;
    }
    if (staged && !c->staged_ok)
        return fail(c, TLSPH_E_UNSUPPORTED,
                    "the LDS-staged force pass does not fit this input at this tile size");
    if (blk_a <= 0) {
        tlsph_status ts = set_tile_a(c, blk_a == 0 ? c->st.tile : -blk_a, stream);
        if (ts != TLSPH_OK) return ts;
        if (!c->st.staged_lds_a)
            return fail(c, TLSPH_E_UNSUPPORTED, "the staged deformation pass does not fit LDS");
    }
    c->st.staged = staged;
    c->sub_b = sub;
    c->block_b = staged ? c->st.tile * sub : blk_b;
    c->block_a = blk_a > 0 ? blk_a : 0;
    return TLSPH_OK;
}

void tlsph_destroy(tlsph_ctx* c) {
    if (!c) return;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
