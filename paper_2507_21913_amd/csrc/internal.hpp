// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fmmhp.h"
#include "cplx.hpp"

namespace fmmhp {

constexpr int kLBits = 30;        // integer cell bits per axis of the root square
constexpr int kLBitsForest = 27;  // the same in a forest (instance index in the top key bits)
constexpr int kMaxInstances = 512;
constexpr int kVecChunk = 8;        // charge vectors evaluated together
constexpr int kNearHeavyGroups = 8; // near-field workgroups per CU at least, for gradient and dipole passes
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;  // device scratch of fmmhp_eval_noalloc
constexpr int64_t kSurfChunk = 2048;  // points per partial sum of the surface term
constexpr double kMaxTablePZ = 24.0;   // |Z| * distance covered by the M2L tables
constexpr double kMaxDevicePZ = 12.0;  // the same for the device-side I_n recursion (W, X lists)
constexpr int kTile = 64;         // target boxes per M2L tile (one per lane)
constexpr int kNumSlots = 49;     // 7 x 7 same-level offsets, |dx|, |dy| <= 3
constexpr int kNumImgSlots = 21;  // image offsets: dx in [-3, 3], dy in {-3, -2, -1}
constexpr int kM2LChunkMax = 8;   // at most this many output coefficients per M2L wave
constexpr int kM2LPhase = 4;      // multipole coefficients staged in LDS per phase
constexpr int kM2LMaxSrc = 400;   // distinct V sources per tile (LDS: 4 * 400 * 16 B)

// Waves per M2L workgroup, each owning m2l_chunk(PB) consecutive output coefficients: the fewest
// waves of at most kM2LChunkMax outputs, with the outputs spread evenly over them.
__host__ __device__ constexpr int m2l_waves(int PB) { return (PB + kM2LChunkMax) / kM2LChunkMax; }
__host__ __device__ constexpr int m2l_chunk(int PB) { return (PB + m2l_waves(PB)) / m2l_waves(PB); }

// Matrix-core FP64 M2L: column blocks of 16 embedded outputs (8 complex coefficients each) and steps
// of 4 complex source coefficients.
__host__ __device__ constexpr int mf_ncb(int PB) { return (2 * (PB + 1) + 15) / 16; }
__host__ __device__ constexpr int mf_nks(int PB) { return (PB + 4) / 4; }

// M2L operator rows are zero-padded so that every reader stays in bounds: the vector kernel's chunks
// read up to m2l_waves(PB) * m2l_chunk(PB) + PB entries, the matrix-core kernel's padded
// (output, source) coefficient pairs up to index 8 mf_ncb(PB) + 4 mf_nks(PB) - 2.
__host__ __device__ constexpr int m2l_row(int PB) {
    return m2l_waves(PB) * m2l_chunk(PB) + PB > 8 * mf_ncb(PB) + 4 * mf_nks(PB) - 1
               ? m2l_waves(PB) * m2l_chunk(PB) + PB
               : 8 * mf_ncb(PB) + 4 * mf_nks(PB) - 1;
}

void set_error(const char *fmt, ...);

#define FMMHP_HIP(expr)                                                              \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::fmmhp::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                                 \
            return FMMHP_EHIP;                                                       \
        }                                                                            \
    } while (0)

#define FMMHP_CHECK(expr)                    \
    do {                                     \
        fmmhp_status s_ = (expr);            \
        if (s_ != FMMHP_OK) return s_;       \
    } while (0)

// Device allocations owned by one plan.
struct Arena {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    fmmhp_status alloc(void **p, size_t nbytes, const char *what);
    template <class T>
    fmmhp_status alloc_n(T **p, size_t n, const char *what) {
        return alloc((void **)p, (n ? n : 1) * sizeof(T), what);
    }
    void release();
};

struct Tree {
    int64_t n = 0;
    int depth = 0;
    int nbox = 0, nleaf = 0;
    double x_lo = 0, S = 0, scale = 0;  // root square of instance 0
    int n_inst = 1;
    int lbits = kLBits;
    std::vector<int64_t> inst_off;      // [n_inst + 1] point ranges of the instances
    std::vector<double> inst_xlo, inst_S, inst_scale;
    int32_t *inst = nullptr;            // box -> instance
    std::vector<int> lev_start;   // boxes of level l: [lev_start[l], lev_start[l + 1]), l >= 1
    // sorted points
    double *xs = nullptr, *ys = nullptr;
    int32_t *perm = nullptr;      // sorted position -> input index
    int32_t *leaf_of = nullptr;   // sorted position -> leaf box
    // boxes
    int32_t *level = nullptr, *bx = nullptr, *by = nullptr, *first = nullptr, *count = nullptr;
    int32_t *parent = nullptr, *leaf = nullptr, *child_first = nullptr, *nchild = nullptr;
    uint64_t *prefix = nullptr;   // Morton prefix at the box's level (sorted within a level)
    // lists (0 U, 1 V, 2 W, 3 X), CSR with int32 offsets
    int32_t *off[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *ent[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t len[4] = {0, 0, 0, 0};
};

// Points from src_end on are target-only (they carry no charge; y = 0 allowed).
fmmhp_status build_tree(Arena &A, Tree &T, int n_inst, const int64_t *inst_off, const double *x, const double *y,
                        const double *img_x, const double *img_y, int64_t src_end, int leaf_size, int max_level,
                        hipStream_t stream);

// Root square and impedance of one instance of a plan.
struct InstInfo {
    double x_lo, S;
    cplx Z;
    double isg;      // sign of the image log term: +1 (Robin, Dirichlet) or -1 (Neumann)
    int32_t react;   // 1: the reaction term G_Z is present (Robin); 0: Dirichlet or Neumann
    int32_t pad;
};

// A range of sorted points within one instance.
struct PtChunk {
    int64_t start, end;
    int32_t inst, pad;
};

// Adjoint workspace, allocated on the first backward call.
struct BwdWork {
    bool ready = false;
    double *q3 = nullptr;                 // [3][n] q, Re conj(g), Im conj(g) (caller order)
    double *qc = nullptr;                 // [n] coincident charge sums of q (sorted order)
    cplx *phi3 = nullptr;                 // [3][n] potentials (caller order)
    cplx *gx3 = nullptr, *gy3 = nullptr;  // [3][n] gradients (caller order)
    cplx *near_gx = nullptr, *near_gy = nullptr;  // [3][n] near-field gradients (sorted order)
    cplx *red = nullptr;                  // [n chunks + n_inst] reduction partials + results
};

// Per-vector workspace of an evaluation pass over up to cap charge vectors.
struct VecWs {
    int cap = 0;
    cplx *W = nullptr;              // [nv][PB + 1][nbox] multipoles
    cplx *Lam = nullptr;            // [nv][nloc][PB + 1][nbox] locals
    double *qs = nullptr;           // [n][nv] sorted charges, vectors interleaved
    double2 *near = nullptr;        // [nv][n] near-field sums
    cplx *red = nullptr;            // [nv][n_rch] surface partial sums
    cplx *rank1 = nullptr;          // [nv][n_inst] surface sums
    float *Wf = nullptr;            // [nv][nbox][KP] FP32 source rows of the matrix-core M2L
    double *part = nullptr;         // [partial entries][nv] column sums of the symmetric near-field walk
};

// Evaluation schedule and tables derived from the tree.
struct Sched {
    int PB = 0;                     // compiled truncation order
    int bc = 0;                     // boundary condition: 0 Robin, 1 Dirichlet, 2 Neumann
    bool real_Z = true;
    cplx Z{0, 0};
    int nloc = 1;                   // 1: H only (real impedance); 2: H and G
    // M2L
    int32_t *vimg_off = nullptr;    // [nbox + 1]  image V entries per box
    int32_t *vimg_ent = nullptr;    // (src << 5) | img_slot
    int nibox = 0;
    int32_t *ibox = nullptr;        // boxes with image V entries
    int ntiles = 0;
    int32_t *tiles = nullptr;       // [ntiles][kTile] box ids (-1 padding)
    int32_t *tile_level = nullptr;  // [ntiles]
    int32_t *tile_src_off = nullptr;  // [ntiles + 1] distinct upper V sources of each tile
    int32_t *tile_src = nullptr;
    int16_t *tile_slot = nullptr;   // [ntiles][kNumSlots][kTile] index into the tile's sources, -1
    uint64_t *tile_mask = nullptr;  // [ntiles] slots used by any lane of the tile
    // X list targets
    int nxbox = 0;
    int32_t *xbox = nullptr;
    int32_t *leaves = nullptr;      // [nleaf]
    int64_t n_wpts = 0;
    int32_t *wpts = nullptr;        // sorted points whose leaf has a W list
    int64_t n_rpts = 0;
    int32_t *rpts = nullptr;        // sorted points whose leaf has image U entries
    int2 *u2 = nullptr;             // [U entries] (first point, count | image << 31) of the source box
    double2 *xy = nullptr;          // [n] sorted (x, y) pairs
    double2 *logtab = nullptr;      // near-field log table
    hipStream_t side = nullptr;     // side stream for the near field (default priority)
    hipStream_t side2 = nullptr;    // second side stream: M2L of the deep levels (default priority)
    hipEvent_t ev_deep_ready = nullptr, ev_deep_done = nullptr;
    int deep_level = 0;             // first level of the deep M2L part (0: no split)
    std::vector<int> tile_lev, ibox_lev;  // per-level ranges of tiles and image-V boxes
    int cus = 1;                    // compute units of the device
    int near_walk = 1;              // near-field walk: 1 prefetching, 2 plain, 3 symmetric leaf pairs
    // symmetric leaf-pair walk (potential passes): leaves with a U list, their jobs, gather lists
    bool sym_ok = false;
    bool sym_built = false;  // the symmetric walks' schedule has been built (on first use)
    int sym_nrec = 0;
    int64_t sym_npart = 0;          // partial-sum entries per vector
    int4 *sym_rec = nullptr;        // (first target, targets, first job, end of jobs) per record
    int4 *sym_jobs = nullptr;       // (first point of B, count | image << 31, partial slot or -1, 0)
    int32_t *sym_in_off = nullptr, *sym_in = nullptr;  // per box: its partial slots (gather)
    int64_t near_blocks = 512;      // near-field grid (workgroups)
    bool fork_late = false;         // start the deep M2L after the whole upward pass
    bool serial = false;            // every kernel on the eval stream (FMMHP_FLAG_SERIAL)
    bool rank1_side = true;         // surface sums on the near-field stream
    int sub_level = 0;              // cut level of the subtree M2M / L2L passes (0: one launch per level)
    int n_sub = 0, sub_nlev = 0;    // subtrees (the boxes of the cut level), levels cut..depth
    int2 *sub_rng = nullptr;        // [n_sub][sub_nlev] box range of each subtree per level
    int sub_ld_m2m = 0, sub_ld_l2l = 0;  // LDS expansion slots of the subtree passes
    // subtrees below the cut too large for those slots: parent (M2M) and child (L2L) chunks by level
    int2 *m2m_ch = nullptr, *l2l_ch = nullptr;
    // P2L groups: {first X box (index into xbox), X sources of the group, first entry of xgent, 0},
    // one sentinel {nxbox, 0, entries, 0}; groups never cross a level (xgrp_lev[l] = first group of
    // level l).  xgent: {list entry code, box slot in the group, first row in the group, first
    // source point}; xgeo: per X box {centre x, centre y, half side, instance}
    int4 *xgrp = nullptr, *xgent = nullptr;
    double4 *xgeo = nullptr;
    std::vector<int> xgrp_lev;
    std::vector<int> m2m_ch_lev, l2l_ch_lev;  // [depth + 2] first chunk of each level
    // L2L of levels 4..cut in one launch: subtrees rooted at level 3 (0 subtrees: one launch per level)
    int n_top = 0, top_nlev = 0, top_ld_l2l = 0, top_ld_m2m = 0;  // (the same subtrees serve the M2M)
    int2 *top_rng = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_up = nullptr;  // upward pass done (main stream)
    // tables
    cplx *Tfree = nullptr;          // [kNumSlots][m2l_row(PB)]
    bool m2l_fp32 = false;          // FMMHP_FLAG_M2L_FP32: upper-source M2L on the FP32 matrix cores
    int m2l_form = 0;               // FP64 M2L of upper sources: 0 default (vector ALUs), 1 vector ALUs
                                    // (k_m2l), 2 matrix cores (k_m2l_mf)
    float *Bf32 = nullptr;          // [kNumSlots][KP][NP] embedded scaled operators (FP32 M2L)
    cplx *Lfree = nullptr;          // [kNumSlots]   (offset part of the log term)
    cplx *TimgH = nullptr;          // [blocks][kNumImgSlots][m2l_row(PB)]
    cplx *TimgG = nullptr;          // same, G-local (complex impedance only)
    cplx *Limg = nullptr;           // [kNumImgSlots]
    double *logside = nullptr;      // [nbox] log(2 rho) of each box
    int32_t *ibase = nullptr;       // [nbox] image-table block of the box's (instance, level), or -1
    InstInfo *inst_info = nullptr;  // [n_inst]
    cplx *E_m2m = nullptr;          // [4][PB + 1]  (-eps)^j / j!
    cplx *E_l2l = nullptr;          // [4][PB + 1]  eps^j / j!
    double *invfact = nullptr;      // [2 PB + 2]
    double *fact = nullptr;         // [2 PB + 2]
    // surface-term chunks
    int n_rch = 0;
    PtChunk *rch = nullptr;         // [n_rch]
    int32_t *inst_ch = nullptr;     // [n_inst + 1] chunk range of each instance
    VecWs ws;                       // workspace of the plan's own evaluations
    BwdWork bw;
    double *cq = nullptr, *cphi = nullptr;  // complex-charge workspace ([2][n], [2][n][2])
    double2 *nrm = nullptr;         // [n] source normals in sorted order (double-layer evaluation)
    // recorded evaluation (FMMHP_FLAG_GRAPH)
    bool use_graph = false;
    struct {
        hipGraphExec_t exec = nullptr;
        const double *q = nullptr;
        double *phi = nullptr;
        int nvec = 0;
        hipStream_t stream = nullptr;
    } graph;
    // algorithmic work counts
    int64_t p2p_pairs[2] = {0, 0};
    int64_t m2l_pairs[2] = {0, 0};
    // phase timing (profiling aid)
    bool timing = false;
    std::vector<hipEvent_t> *events = nullptr;   // per timed pass: phase boundaries, near, deep, k_m2l pairs
    std::vector<int> *m2l_n = nullptr;            // per timed pass: k_m2l launches (0, 1 or 2)
    double phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t timed_evals = 0;
    double m2l_kernel_ms = 0.0;                   // summed k_m2l launch durations since timing was enabled
    int64_t m2l_launches = 0;
};

// Zs: [T.n_inst] impedance of each instance (host)
fmmhp_status build_schedule(Arena &A, const Tree &T, Sched &S, int PB, const cplx *Zs, hipStream_t stream);
fmmhp_status apply_launch_shape(Arena &A, const Tree &T, Sched &S, int near_walk, int near_groups, hipStream_t s);
fmmhp_status run_eval(Arena &A, const Tree &T, Sched &S, int nvec, const double *q, double *phi,
                      hipStream_t stream);
// The same evaluation with each pass's workspace in the library's static device scratch (no
// allocation); device is the plan's device, which must be current.
fmmhp_status run_eval_noalloc(const Tree &T, const Sched &S, int device, int nvec, const double *q, double *phi,
                              hipStream_t stream);
// Double-layer potential of nvec dipole densities mu ([nvec][n], w = 1 real or 2 complex) with
// source normals nx, ny [n], all in caller order.
fmmhp_status run_eval_dlp(Arena &A, const Tree &T, Sched &S, int nvec, const double *mu, int w, const double *nx,
                          const double *ny, double *phi, hipStream_t s);
fmmhp_status run_eval_complex(Arena &A, const Tree &T, Sched &S, int nvec, const double *q, double *phi,
                              hipStream_t stream);

fmmhp_status run_field(Arena &A, const Tree &T, Sched &S, const double *q, double *phi, cplx *gx, cplx *gy,
                       hipStream_t stream);
// Clears n doubles on stream with a kernel (no memset node under graph capture).
fmmhp_status zero_f64(double *p, int64_t n, hipStream_t stream);

// zsum_host: per-instance homogeneity sums copied to the host (the call synchronises), or null;
// dlz_dev: (dl/dRe Z_k, dl/dIm Z_k) written on the device instead (no synchronisation), or null.
fmmhp_status run_backward(Arena &A, const Tree &T, Sched &S, const double *q, const double *g, double *grad_q,
                          double *grad_x, double *grad_y, cplx *zsum_host, double *dlz_dev, hipStream_t stream);

fmmhp_status collect_phase_times(Sched &S);
fmmhp_status run_direct(int64_t ns, const double *sx, const double *sy, int nvec, const double *q,
                        int64_t nt, const double *tx, const double *ty, cplx Z, double *phi,
                        hipStream_t stream);
fmmhp_status run_reaction_integrals(int64_t m, const double *x, const double *y, int nmax, cplx Z,
                                    double *out, hipStream_t stream);

inline int pick_bucket(int p) {
    int b = ((p + 4) / 5) * 5;
    return b < 5 ? 5 : b;
}

}  // namespace fmmhp

struct fmmhp_plan_s {
    uint64_t magic;
    int device;
    // separate targets (fmmhp_plan_create_targets): points [0, n_src) are the sources, the rest
    // target-only; 0 when sources are the targets.  Evaluation pads the charges with zeros and
    // keeps the targets' potentials.
    int64_t n_src = 0;
    double *qpad = nullptr, *phipad = nullptr;  // [cap][n] (x2 for complex charges), [cap][n][2]
    double *gpad = nullptr;                     // [2][n][2] gradients at all points (fmmhp_eval_field)
    double *npad = nullptr;                     // [2][n] normals padded to all points (double layer)
    double *ndwork = nullptr;                   // [3][n_tgt][2] field at the targets (normal derivative)
    int pad_cap = 0;
    int p_req, leaf_size, max_level;
    double lambda_re, lambda_im;
    std::vector<fmmhp::cplx> Zs;  // impedance of each instance
    fmmhp::Arena arena;
    fmmhp::Tree tree;
    fmmhp::Sched sched;
};
