// Host-side structures of the library and the launchers the C ABI calls.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mad.h"
#include "mlp.hpp"

struct mad_mesh {
    int64_t nv = 0, nt = 0;
    std::vector<int32_t> tris;           // [nt][3]
    std::vector<int64_t> comp_off;       // [ncomp + 1]; {0, nv} when not batched
    bool batched = false;
    // topology (built at create): edges sorted by (min, max)
    std::vector<int32_t> edges;          // [ne][2]
    std::vector<int32_t> edge_nf;        // [ne] incident face count
    std::vector<int32_t> edge_face0;     // [ne] lowest incident face
    std::vector<int32_t> diamonds;       // [nd][4]
    std::vector<int32_t> diamond_faces;  // [nd][2]
    std::vector<int32_t> vert_face0;     // [nv] lowest face containing the vertex (-1: none)
    // face adjacency across manifold and non-manifold edges (CSR), for patching
    std::vector<int32_t> fadj_ptr, fadj;
    int64_t ne() const { return (int64_t)edge_nf.size(); }
    int64_t nd() const { return (int64_t)diamond_faces.size() / 2; }
};

namespace mad {

struct Term {
    int kind = 0;
    int ns = 0, d = 0, nrest = 0;
    double prm[4] = {0, 0, 0, 0};
    int64_t n = 0;
    std::vector<int32_t> stencil;        // original order [n][ns]
    std::vector<double> rest;            // original order [n][nrest]
    std::vector<int32_t> elem_patch;     // patch of each element (original order)
    // patch-ordered device data
    std::vector<int32_t> perm;           // device slot -> original element
    std::vector<int32_t> elem_ptr;       // [n_patch + 1]
    int32_t* d_stencil = nullptr;        // [n][ns]
    double* d_rest = nullptr;            // SoA [nrest][n]
    int32_t* d_elem_ptr = nullptr;       // [n_patch + 1]
    int32_t* d_slots = nullptr;          // SoA [ns*ns][n] global block of (s, t) (atomic scatter)
    uint16_t* d_lvert = nullptr;         // SoA [ns][n] patch-local vertex (patch scatter)
    uint16_t* d_lslot = nullptr;         // SoA [ns(ns+1)/2][n] patch-local block + flags
    uint8_t* d_lseg = nullptr;           // [n] segment of the element inside its 64-element work unit
    const mad_mlp* mlp = nullptr;        // learned density: the network
    float* d_psi = nullptr;              // learned density: SoA [28][n] network outputs, patch order
    float* d_xh = nullptr;               // learned density: SoA [6][n] scaled features, patch order
    const double* vdata = nullptr;       // vertex terms: the caller's [nv][NVD] device array (not owned)
    int32_t* d_jstencil = nullptr;       // residual terms: [n][ns] in element order (the rows' owners)
    double* d_jrest = nullptr;           // residual terms: SoA [nrest][n] in element order
    // colored scatter: elements sorted by color; elem_ptr then delimits chunks of at most kColorChunk elements
    // of one color and one component, color_chunk_ptr[c] is the first chunk of color c, and d_slot_map gives
    // each chunk's energy slot (slots ordered by component, then term, color and chunk)
    std::vector<int32_t> color_chunk_ptr;
    std::vector<int32_t> slot_map;       // host copy of d_slot_map
    int32_t* d_slot_map = nullptr;
};

// patch-local index structures of the LDS-accumulating assembly (host_patch.cpp)
struct PatchLocal {
    std::vector<int32_t> lv_ptr, lv_global;          // per patch: touched vertices (sorted)
    std::vector<int32_t> lv_halo;                    // -1: vertex touched by this patch only; else halo slot
    std::vector<int32_t> lb_ptr, lb_gidx, lb_gidxT;  // per patch: upper blocks (r <= c): (r,c), (c,r)
    std::vector<int32_t> lb_halo;                    // -1: block touched by this patch only; else halo slot
    std::vector<std::vector<uint16_t>> lvert;        // per term, SoA [ns][n] local vertex
    std::vector<std::vector<uint16_t>> lslot;        // per term, SoA [ns(ns+1)/2][n] local block + flags
    // gather of shared entries: per shared vertex / upper block, its halo slots in patch order
    std::vector<int32_t> gv_ptr, gv_src, gv_vert;
    std::vector<int32_t> gb_ptr, gb_src, gb_gidx, gb_gidxT;
    std::vector<int32_t> orphan_vert, orphan_block; // entries no patch touches (isolated vertices)
    int32_t max_lv = 0, max_lb = 0;
};

// one contiguous range of patches per component
struct Patches {
    int32_t n = 0;
    std::vector<int32_t> face_patch;     // [nt]
    std::vector<int32_t> comp_patch_ptr; // [ncomp + 1]
};

// scratch of the pattern update for new interaction pairs, sized at finalize from the reserve
struct DynBuffers {
    int32_t* cnt = nullptr;      // [nv + 1] candidate blocks per row
    int32_t* fill = nullptr;     // [nv + 1]
    int32_t* coff = nullptr;     // [nv + 1] candidate offsets
    int32_t* stage = nullptr;    // [2 * max_pairs] candidate columns, by row
    int32_t* nnew = nullptr;     // [nv] distinct new blocks per row
    int32_t* rowcnt = nullptr;   // [nv] new row lengths
    int32_t* noff = nullptr;     // [nv + 1]
    int32_t* map = nullptr;      // [capacity] old block -> new block
    int32_t* flags = nullptr;    // [4]
    int64_t* rp64 = nullptr;     // [nv + 1]
    int64_t* scan_tmp = nullptr;
};

}  // namespace mad

struct mad_problem {
    const mad_mesh* mesh = nullptr;
    int d = 0, prec = 0;
    mad_options opt{};
    std::vector<mad::Term> terms;
    bool finalized = false;
    int device = 0;
    mad::Patches patches;
    int64_t nnzb = 0;
    int32_t* d_rowptr = nullptr;          // the active pattern buffer
    int32_t* d_colidx = nullptr;
    // dynamic sparsity (interaction pairs): a second pattern buffer, both of capacity nnzb_cap; the blocks
    // added since the last layout build, which no term touches and every Hessian evaluation zeroes
    int64_t pair_reserve = 0;             // max pairs per insertion (0: no insertion)
    int64_t nnzb_cap = 0;
    int32_t* d_rowptr_b = nullptr;
    int32_t* d_colidx_b = nullptr;
    int32_t* d_extra_blocks = nullptr;    // [2 * pair_reserve]
    int64_t n_extra = 0;
    bool host_pattern_stale = false;      // h_rowptr / h_colidx lag the device pattern
    mad::DynBuffers dyn;
    int64_t n_lb = 0;                     // entries of d_lb_gidx / d_lb_gidxT
    int32_t* d_comp_patch_ptr = nullptr;
    double* d_partial = nullptr;          // [n_terms][n_patch]
    double* d_comp_energy = nullptr;      // [n_comp] per-component energies (reduction scratch)
    int32_t* d_flags = nullptr;           // [0] nonfinite, [1] internal-error bits (kFlag*)
    unsigned long long* d_fallbacks = nullptr;
    int scatter = MAD_SCATTER_PATCH;
    int persistent = 0;                   // patch scatter: persistent grid pulling patches from a queue
    int wg_waves = 4;                     // patch scatter tile: waves per workgroup (4, or 8 with FP32)
    int n_cu = 0;                         // compute units of the device
    std::vector<void*> layout_owned;      // device memory of the current layout (freed on relayout)
    std::vector<int32_t> h_rowptr, h_colidx;  // host copy of the pattern (layout rebuilds)
    int32_t* d_color_comp_ptr = nullptr;  // colored scatter: [n_comp + 1] energy slots of each component
    int64_t n_color_slots = 0;            // colored scatter: energy slots (chunks of all terms)
    int32_t* d_work_order = nullptr;      // patches, largest first (persistent launch)
    int32_t* d_work_counter = nullptr;
    std::string tune_report;              // last autotune table (JSON)
    bool shell = false;                   // a term reads the shell features (needs vertex normals)
    bool light = true;                    // every term is a spring, inertia, edge-length or residual term
    int32_t* d_tris = nullptr;            // [nt][3] mesh triangles (normals)
    int32_t* d_vf_ptr = nullptr;          // [nv + 1] vertex -> triangles, ascending
    int32_t* d_vf = nullptr;
    double* d_normals = nullptr;          // [nv][3] unit vertex normals of the evaluated positions
    int32_t* d_lv_ptr = nullptr;
    int32_t* d_lv_global = nullptr;
    int32_t* d_lv_halo = nullptr;
    int32_t* d_lb_ptr = nullptr;
    int32_t* d_lb_gidx = nullptr;
    int32_t* d_lb_gidxT = nullptr;
    int32_t* d_lb_halo = nullptr;
    int32_t* d_gv_ptr = nullptr;
    int32_t* d_gv_src = nullptr;
    int32_t* d_gv_vert = nullptr;
    int32_t* d_gb_ptr = nullptr;
    int32_t* d_gb_src = nullptr;
    int32_t* d_gb_gidx = nullptr;
    int32_t* d_gb_gidxT = nullptr;
    int32_t* d_orphan_vert = nullptr;
    int32_t* d_orphan_block = nullptr;
    int32_t n_gv = 0, n_gb = 0, n_orphan_vert = 0, n_orphan_block = 0;
    void* d_halo_g = nullptr;             // [halo vertex slots][D] partial gradients of shared vertices
    void* d_halo_h = nullptr;             // [halo block slots][D*D] partial blocks of shared blocks
    void* d_halo_y = nullptr;             // [halo vertex slots][D] partial Hessian-vector products
    int64_t n_halo_v = 0, n_halo_b = 0;   // halo slots of shared vertices / shared upper blocks
    uint32_t* d_fb_list = nullptr;
    int32_t* d_fb_count = nullptr;
    int32_t fb_cap = 0;
    size_t lds_bytes = 0;
    int32_t max_lv = 0, max_lb = 0;
    std::vector<void*> owned;             // every device allocation, freed at destroy
    // profiling: one row of n_terms + 3 events per recorded evaluation
    bool profiling = false;
    int64_t prof_count = 0;
    std::vector<std::vector<hipEvent_t>> prof_events;
};

namespace mad {

// bits of a problem's internal-error flag word (d_flags[1]); mad_problem_status turns any into MAD_E_INTERNAL
constexpr int32_t kFlagSlotMissing = 4;        // atomic scatter: an element block is not in the pattern
constexpr int32_t kFlagRedoBlockMissing = 8;   // FP64 redo: an element block is not in the pattern
constexpr int32_t kFlagLockTimeout = 16;       // patch kernel: a wait for the LDS lock reached its bound
constexpr int32_t kFlagQueueOverflow = 32;     // more FP32 elements queued for the FP64 redo than the queue holds
constexpr int32_t kDefaultLockSpins = 1 << 22;

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define MAD_HIP_TRY(expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return ::mad::fail(MAD_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int kind_stencil(int kind);
int kind_vardim(int kind);
int kind_nrest(int kind);

// host setup (host_mesh.cpp)
int build_topology(mad_mesh& m);
int rest_tri(const mad_mesh& m, const double* rest_pos, std::vector<double>& out);        // [nt][5]
int rest_diamond(const mad_mesh& m, const double* rest_pos, std::vector<double>& out);    // [nd][2]
int rest_shell(const mad_mesh& m, const double* rest_pos, std::vector<double>& out);      // [nt][8]
int rest_spring(const mad_mesh& m, const double* rest_pos, std::vector<double>& out);     // [ne][2]
int rest_edge_length(const mad_mesh& m, const double* rest_pos, std::vector<double>& out);  // [ne]
void build_patches(const mad_mesh& m, int target_faces, Patches& p);
// host_layout.cpp: element order by patch, colour order inside patches, the largest patch's vertex and
// upper-block counts, segments of the 64-element work units
void order_terms(mad_problem* p);
void color_within_patches(Term& t, int64_t nv);
void patch_extent(const mad_problem* p, int32_t* max_lv, int32_t* max_lb);
void unit_segments(const Term& t, int32_t np, int64_t nv, std::vector<uint8_t>& seg);
// colored scatter: greedy coloring of each term's elements (no shared vertex within a color), elements
// sorted by color then component, chunks, energy slots; comp_slot_ptr [n_comp + 1] (host)
constexpr int kColorChunk = 256;
void color_order(mad_problem* p, std::vector<int32_t>& comp_slot_ptr);
// layout.cpp: (re)build the element order and the scatter structures of a problem
int build_layout(mad_problem* p, int target_faces, int scatter, int persistent, hipStream_t s, int wg_waves = 0);
int build_scatter(mad_problem* p, hipStream_t s);
// Device buffers an evaluation writes and reads back within itself; nothing in them outlives the
// evaluation. By default the problem's own (allocated with its layout); mad_problem_eval_static takes
// them from the library's static scratch array instead.
struct EvalScratch {
    double* partial = nullptr;        // [n_terms][n_patch] per-patch energies
    double* comp_energy = nullptr;    // [n_comp] per-component energies (reduction scratch)
    int32_t* work_counter = nullptr;  // head of the persistent launch's patch queue
    int32_t* fb_count = nullptr;      // length of the FP64 redo queue
    uint32_t* fb_list = nullptr;      // [fb_cap] FP32 elements queued for the FP64 redo
    int32_t fb_cap = 0;
    void* halo_g = nullptr;           // [n_halo_v][D]
    void* halo_h = nullptr;           // [n_halo_b][D*D]
    void* halo_y = nullptr;           // [n_halo_v][D] (matrix-free products only)
    double* normals = nullptr;        // [nv][3] unit vertex normals (shell-feature terms)
    float* psi[8] = {};               // per term: network outputs SoA [28][n] (learned density)
    float* xh[8] = {};                // per term: scaled features SoA [6][n] (learned density)
};
EvalScratch own_scratch(const mad_problem* p);
// argument checks shared by mad_problem_eval and mad_problem_eval_static
int check_eval_args(const mad_problem* p, const double* x, uint32_t mode, const double* energy, const void* grad,
                    const void* hess);
// one evaluation; with v != NULL the matrix-free product y = H v replaces the Hessian (hess NULL);
// sc NULL: the problem's own scratch
int eval_problem(mad_problem* p, const double* x, uint32_t mode, double* energy, void* grad, void* hess,
                 hipStream_t s, const double* v = nullptr, void* y = nullptr, const EvalScratch* sc = nullptr);
constexpr size_t kLdsBudget = 76 * 1024;  // dynamic LDS per workgroup: two workgroups in a CU's 160 KB
// the whole CU's LDS but its static part, for the 8-wave tile of heavy terms (one workgroup per CU: two waves
// per SIMD are all their registers allow)
constexpr size_t kLdsBudgetWide = 148 * 1024;
// the LDS budget of a problem's current tile
size_t lds_budget(const mad_problem* p);
// work units (64 elements of one term) per patch: the patch kernel keeps one energy slot per unit
constexpr int kMaxPatchUnits = 256;
int build_patch_local(mad_problem& P, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& colidx,
                      PatchLocal& L);
size_t patch_lds_bytes(int var_dim, int prec, int mode, int32_t max_lv, int32_t max_lb, bool hvp = false);

// device launchers (kernels_*.hip); all asynchronous on `stream`
struct EvalLaunch {
    int kind;
    int prec;       // MAD_F64 / MAD_F32
    int mode;       // 0 passive, 1 grad, 2 hess, 3 clamped hess
    int want_grad;
    int n_patch;
    const double* x;
    const int32_t* stencil;
    const double* rest;
    int64_t n;      // elements (rest/slot SoA stride)
    const int32_t* elem_ptr;
    const int32_t* slots;
    void* grad;
    void* hess;
    double* partial;
    int32_t* flags;
    unsigned long long* fallbacks;
    double prm[4];
    double eps;
    double qmin;
    const double* normals;  // [nv][3] unit vertex normals (shell-feature terms)
    const float* psi;       // SoA [28][n] network outputs (learned density)
    const double* vdata;    // [nv][NVD] caller's per-vertex data (vertex terms)
    int hvp;                // matrix-free mode: atomically add H_j v_j to y
    const double* v;
    void* y;
    int plain;              // colored scatter: plain read-add-writes (no two elements of the launch share a vertex)
    int chunk0;             // colored scatter: first chunk (workgroup p handles chunk chunk0 + p)
    const int32_t* slot_map;  // colored scatter: energy slot of each chunk (NULL: slot = chunk)
};
hipError_t launch_eval(const EvalLaunch& L, hipStream_t s);

// fused patch kernel: every term of a patch in one workgroup, LDS accumulation, one flush
struct PatchTermArgs {
    int kind;
    int64_t n;
    const double* rest;
    const uint16_t* lvert;
    const uint16_t* lslot;
    const uint8_t* lseg;     // segment inside the work unit (vertex-disjoint elements share one)
    const int32_t* elem_ptr;
    const float* psi;        // SoA [28][n] network outputs (learned density)
    const double* vdata;     // [nv][NVD] caller's per-vertex data (vertex terms)
    double prm[4];
};
struct PatchLaunch {
    int prec, mode, want_grad, var_dim, n_terms, n_patch;
    size_t lds_bytes;
    const double* x;
    void* grad;
    void* hess;
    const int32_t* lv_ptr;
    const int32_t* lv_global;
    const int32_t* lv_halo;
    const int32_t* lb_ptr;
    const int32_t* lb_gidx;
    const int32_t* lb_gidxT;
    const int32_t* lb_halo;
    void* halo_g;
    void* halo_h;
    double* partial;
    int32_t* flags;
    unsigned long long* fallbacks;
    uint32_t* fb_list;      // queued FP32 elements: term << 29 | element
    int32_t* fb_count;
    int32_t fb_cap;
    double eps, qmin;
    const double* normals;  // [nv][3] unit vertex normals (shell-feature terms)
    int shell;              // the problem has shell-feature terms (selects the kernel variant)
    int light;              // every term is a light term (edge, spring, vertex, residual): the light variant
    int term_order[8];      // terms by decreasing element cost (work units of the costliest first)
    int hvp;                // matrix-free mode: y = H v instead of assembling H (modes 2, 3)
    const double* v;        // [nv][D]
    void* y;                // [nv][D], T
    void* halo_y;           // [halo vertex slots][D] partial products of shared vertices
    int lock_spins;         // bound on each LDS-lock wait (0: give up at once)
    int persistent;
    int block;              // threads per workgroup: 256, or 512 (FP32 only)
    const int32_t* work_order;
    int32_t* work_counter;
    int n_cu;
    PatchTermArgs terms[8];
};
hipError_t launch_eval_patch(const PatchLaunch& L, hipStream_t s);

// sum the halo partials of every shared entry in a fixed order and write it once; zero orphans
struct GatherLaunch {
    int prec, var_dim, want_grad, want_hess;
    void* grad;
    void* hess;
    const void* halo_g;
    const void* halo_h;
    const int32_t *gv_ptr, *gv_src, *gv_vert;
    const int32_t *gb_ptr, *gb_src, *gb_gidx, *gb_gidxT;
    const int32_t *orphan_vert, *orphan_block;
    int32_t n_gv, n_gb, n_orphan_vert, n_orphan_block;
};
hipError_t launch_gather(const GatherLaunch& G, hipStream_t s);

// FP64 redo of the queued FP32 elements, added to the FP32 outputs with atomics
struct FallbackTerm {
    int kind;
    int64_t n;
    const int32_t* stencil;  // [n][ns] global vertices, patch order
    const double* rest;
    const float* psi;
    const double* vdata;
    double prm[4];
};
struct FallbackLaunch {
    int var_dim, want_grad;
    const double* x;
    void* grad;
    void* hess;
    const int32_t* rowptr;
    const int32_t* colidx;
    const uint32_t* fb_list;
    const int32_t* fb_count;
    int32_t fb_cap;
    int32_t* flags;
    double eps;
    const double* normals;
    int hvp;                // add H_j v_j to y instead of H_j to the blocks
    const double* v;
    void* y;
    FallbackTerm terms[8];
};
hipError_t launch_fallback(const FallbackLaunch& F, hipStream_t s);
hipError_t launch_fill(void* ptr, int64_t n_elems, int elem_bytes, hipStream_t s);
// one small kernel that zeroes up to two int32 counters (either may be null)
hipError_t launch_zero_counters(int32_t* a, int32_t* b, hipStream_t s);
hipError_t launch_energy_reduce(const double* partial, int n_terms, int n_patch, const int32_t* comp_patch_ptr,
                                int n_comp, bool batched, double* energy, double* comp_scratch, hipStream_t s);

// pattern builder (kernels_pattern.hip)
struct PatternTerm {
    const int32_t* stencil;  // device [n][ns]
    int64_t n;
    int ns;
};
// Builds rowptr/colidx on the device (allocated here, appended to `owned`); nnzb returned.
int build_pattern_device(int64_t nv, const std::vector<PatternTerm>& terms, int32_t** rowptr, int32_t** colidx,
                         int64_t* nnzb, std::vector<void*>& owned, hipStream_t s);
hipError_t launch_slots(const int32_t* stencil, int64_t n, int ns, const int32_t* rowptr, const int32_t* colidx,
                        int32_t* slots, int32_t* flags, hipStream_t s);
// residual terms: residual vector and row-owned Jacobian (kernels_jac.hip)
struct JacTerm {
    int kind;
    int64_t n;
    const int32_t* stencil;  // [n][ns] global vertices, element order (element e owns its rows)
    const double* rest;      // SoA [nrest][n], element order
    const double* vdata;     // [nv][NVD] caller's per-vertex data
    double prm[4];
    int64_t row_off, nz_off; // the term's first row and first entry
};
struct JacLaunch {
    int prec, pattern, n_terms;
    const double* x;
    double* r;               // [m] FP64
    void* vals;              // [nnz] T
    int32_t* rowptr;         // pattern mode: [m + 1] (the last entry is written by the host)
    int32_t* colidx;         // pattern mode: [nnz]
    int32_t* flags;
    JacTerm terms[8];
};
hipError_t launch_jacobian(const JacLaunch& L, hipStream_t s);
int kind_nres(int kind);

// new interaction pairs [n][2] (device) into the pattern (synchronises the stream)
int insert_pairs_device(mad_problem* p, const int32_t* pairs, int64_t n, int64_t* n_added, hipStream_t s);
// zero the listed blocks (dd values of elem_bytes each)
hipError_t launch_zero_blocks(void* hess, const int32_t* list, int64_t n, int dd, int elem_bytes, hipStream_t s);

}  // namespace mad
