// Internal declarations of libgosma (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gosma.h"

namespace gosma {

struct Solver;   // branch-and-bound buffers (bb.hip)
struct Mlp;      // queue-ordering network (mlp.hip)

// One pose problem as the kernels see it.  Component rows are sorted by class
// label; classes [cls_off, cls_off + n_cls) of the class table list the row
// ranges of each class in both mixtures.
struct ProbDesc {
    int32_t gmm_off, M, vmf_off, N;
    int32_t cls_off, n_cls, bucket, pad1;   // bucket: size bucket of the problem (size_bucket)
    double r_lo[3], r_w[3];     // rotation root box: lo and width
    double t_lo[3], t_w[3];     // translation root box
    double zeta, S22;
};

struct ClassRange {
    int32_t g0, g1, v0, v1;     // absolute row ranges [g0, g1) and [v0, v1)
};

// Device-resident mixtures of every problem.
//   GMM rows: mu (FP64 xyz), 1/sigma^2 (FP64), weight (FP32, see below), and
//   the plain normalised weight used by the branching rule.
//   vMF rows: two float4 per row, {dx, dy, dz, kappa}, {weight, G(kappa),
//   coth(kappa), ln(2 kappa) / 2}, with G(y) = y / (1 - e^{-2y}).
// Weights carry the semantic class weight: with phi_l = 1/|Lambda| and w the
// weights renormalised within the class, the stored weight is sqrt(phi_l) w,
// so the product of two stored weights is phi_l w w' (eq. 17).
struct DevMix {
    const double *mu;
    const double *isig2;
    const float *w1;
    const float *pbar;
    const float4 *vmf;
    const ClassRange *cls;
    const ProbDesc *prob;
    int n_prob;
    // Per-component records of the bound kernels and SMA live in LDS while
    // they fit; for larger mixtures they go to this buffer instead: grec_stride
    // float4 per block, for at most grec_blocks blocks (NULL: LDS).
    float4 *grec;
    int64_t grec_stride;
    int grec_blocks;
    // +infinity, as an argument the compiler cannot fold (see fmin_med3)
    float inf;
};
// Blocks of a bound or SMA launch that stage their records in global memory.
constexpr int kGrecBlocks = 512;
// float4 per block of the global records for mixtures of at most M x N
// components (the largest of the S11, S12 and SMA records).
int64_t grec_stride(int maxM, int maxN);

struct BoundOut {
    double *ub, *lb, *lb_safe, *aux;
    uint8_t *flags;
    float *top8;
    float *psi_gap;    // optional: weighted mean psi_r - weighted mean psi_t (branching statistic)
    unsigned long long *dstar_bits;   // optional: atomic minimum of finite upper bounds (ordered bits),
    int dstar_stride;                 // at dstar_bits[problem * dstar_stride]
    unsigned long long *counts;       // optional work counters (kCountSlots x kCounters, added to; the
                                      // totals are the sums over the slots), see kCnt*
};
// Work counters of timed launches: per slot {live cubes, GMM-vMF pairs
// screened, evaluated, live translation cells, GMM-GMM pairs screened,
// evaluated}; a block adds to slot blockIdx.x % kCountSlots.
constexpr int kCountSlots = 64;
constexpr int kCounters = GOSMA_N_COUNTS;
enum { kCntCubes = 0, kCntS12Screened, kCntS12Evaluated, kCntCells, kCntS11Screened, kCntS11Evaluated };

// A translation-cell key no cell has (the level field of real keys is at most 19).
constexpr uint64_t kEmptyCell = ~0ull;
// launch_s11's out_idx: NULL writes cell c's sums at index c, otherwise at out_idx[c].

// The translation cells of a batch of cubes, deduplicated (the search's cell
// table): 2^tbits slots per problem holding a cell key or kEmptyCell.  The
// set-up pass stores each cube's slot (ctidx, global index) and lists every
// newly claimed cell once (key, problem, slot; count is the list length).
struct CellTable {
    uint64_t *keys;
    uint32_t tbits;
    int64_t *ctidx;
    uint64_t *list_key;
    uint32_t *list_pid;
    int64_t *list_slot;
    uint32_t *count;
};

// Per translation cell and GMM component: the component's quantities that
// depend on the cell alone (the translation part of the per-component set-up
// of the pair kernel).  The GMM-GMM kernel computes them for every distinct
// translation cell of a search iteration and writes them here; the pair
// kernel reads them for each of the cell's cubes instead of recomputing them.
struct alignas(16) TransRec {
    double u[3];                    // (mu - t0) / |mu - t0|
    float kap, klo, ahi, ha;        // kappa at the centre; the interval [klo, ahi], half its width
    float cps, sps, psi;            // cos, sin of psi_t / 2; psi_t (Lemma 3)
    float Gk, cothl, Gl, Gh;        // G(kappa), coth(klo), G(klo), G(ahi)
    float nul, nuh;                 // nu(klo), nu(ahi)
    float lam, ia, hla;             // pair-screen row: ln(w G(ahi)) - ln(klo) / 2, 1 / klo, ln(klo) / 2
    float pad;
};
// The cell's sums over its components: w^2 klo / 2 (the pair screen's
// threshold), the weighted psi_t (branching rule), and its drop flags.
struct alignas(16) CellSums {
    double dk;
    float psum;
    uint32_t flags;   // kCellDrop, kCellUbInf
};
constexpr uint32_t kCellDrop = 1u, kCellUbInf = 2u;
// No record for the cell: the pair kernel computes the values itself.
constexpr uint32_t kNoTRec = 0xffffffffu;
// Offset flag: the cell's record space holds only Lemma 3's half-angle record
// of each component, a float4 {cos, sin of psi_t / 2, psi_t, 0} (written when
// too few cubes share the cells to pay for the full records).
constexpr uint32_t kTRecLemma3 = 0x80000000u;

struct S11Out {
    double *ub, *lo;   // S11 at the centre and its lower bound, per translation cube
    unsigned long long *counts = nullptr;   // optional work counters (see BoundOut)
    // optional per-cell records for the pair kernel (see TransRecs): written
    // at the cell's record offset, which is looked up by its output index
    TransRec *trec = nullptr;
    uint32_t *toff = nullptr;
    CellSums *csum = nullptr;
    // the number of cubes whose pair kernel will read the records: the full
    // records are written only while there are at least kTRecMinCubes cubes
    // per cell, Lemma 3's records otherwise (offsets flagged kTRecLemma3);
    // NULL: always the full records
    const uint32_t *ncubes = nullptr;
};
constexpr int kTRecMinCubes = 8;
// The records of the cells as the pair kernel reads them: the component
// records of a cell at rec[off[cell] + component] (off = kNoTRec: none), its
// sums at csum[cell]; cell indexed like the S11 sums (tidx).
struct TransRecs {
    const TransRec *rec = nullptr;
    const uint32_t *off = nullptr;
    const CellSums *csum = nullptr;
};

// Per-cube set-up of the GMM-vMF pair kernel: both cells decoded, the rotation
// matrix at the rotation cell's centre and the left Jacobian applied to four
// corners of its half-width box.  Uniform across the cube's block, so a small
// kernel computes it once per cube ahead of the pair kernel (one thread per
// cube) instead of every lane of the block; callers of launch_s12 provide
// scratch for one per cube.
struct alignas(16) CubeSetup {
    double R[9];
    double t0[3], tau[3];
    float jc[4][3];
    float hn, cap;       // |h_r| and min(|h_r|, pi)
    uint32_t flags;      // GOSMA_FLAG_DROP_ROT, kSetupPerDir, kSetupInvalid
    uint32_t pad;
};
constexpr uint32_t kSetupPerDir = 0x100u;    // the per-direction Lemma 2 bound applies
constexpr uint32_t kSetupInvalid = 0x200u;   // problem index out of range

// Launch shape of a bound kernel: waves per block (one cell per block; up to
// kMaxWaves) and the number of blocks of the grid-stride loop over cells.
constexpr int kMaxWaves = 4;
struct Tile {
    int waves, blocks;
};

// Problems of a batch are grouped by size into GOSMA_N_BUCKETS buckets, by
// their larger mixture: up to 64, 128, 256 components, and larger.  The
// search bounds each bucket's cubes with a launch of its own, in the launch
// shape tuned for that bucket and with LDS sized for its largest problem.
constexpr int kBuckets = GOSMA_N_BUCKETS;
inline int size_bucket(int M, int N)
{
    const int m = M > N ? M : N;
    return m <= 64 ? 0 : (m <= 128 ? 1 : (m <= 256 ? 2 : 3));
}

// Launchers (bound.hip).  All asynchronous on `stream`.  With a device count
// pointer (nt_dev / n_dev) the kernels read the number of cells from device
// memory (times n_dev_mul); the host count is then the maximum.  Each launch
// runs min(tile.blocks, count) blocks of 64 * tile.waves threads.
hipError_t launch_s11(const DevMix &mx, const uint64_t *tkeys, const uint32_t *pids, int64_t nt, const uint32_t *nt_dev,
                      S11Out out, int maxM, Tile tile, hipStream_t stream, const int64_t *out_idx = nullptr);
hipError_t launch_s12(const DevMix &mx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *pids,
                      const int64_t *tidx, const double *s11ub, const double *s11lo, int64_t n, const uint32_t *n_dev,
                      int n_dev_mul, BoundOut out, double margin_gamma, int maxM, int maxN, bool with_top8, Tile tile,
                      CubeSetup *setup, hipStream_t stream, bool setup_done = false, TransRecs tr = TransRecs{},
                      int kpieces = 1);
// The per-cube set-up pass of k_s12 (and, with cells, the cubes' translation cells).
hipError_t launch_cube_setup(const DevMix &mx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *pids,
                             int64_t n, const uint32_t *n_dev, int n_dev_mul, CubeSetup *setup, const CellTable *cells,
                             hipStream_t stream);
// Dynamic LDS of the two kernels (the pair kernel's grows with the waves per
// block), and the per-kernel limit setup for it.
size_t s11_lds_bytes(int maxM, int waves);
size_t s12_lds_bytes(int maxM, int maxN, int waves, bool vlds);
hipError_t prepare_bound_kernels(int maxM, int maxN);

// SMA (sma.hip): L-BFGS from n starts x0 (n x 6 doubles {r, t}), one block per
// start; results x_out (n x 6), f_out (n), g_out (n x 6 or NULL), it_out (n).
constexpr int kSmaMemory = 5;         // curvature pairs
constexpr double kSmaGtol = 1e-6;     // projected-gradient stop, relative to S11 + 2 S12 at the start
constexpr double kSmaFtol = 1e-9;     // per-step gain stop, relative to |f| + S11 + 2 S12
size_t sma_lds_bytes(int maxM, int maxN);
hipError_t launch_sma(const DevMix &mx, int maxM, int maxN, int64_t n, const uint32_t *pids, const double *x0,
                      int max_iters, int memory, double gtol, double ftol, double *x_out, double *f_out,
                      double *g_out, int32_t *it_out, hipStream_t stream);

// Mixture generation (mixgen.hip): one DP-means (spherical = 0) or
// DP-vMF-means (spherical = 1) clustering with the ML fit of each cluster.
hipError_t dp_cluster(const double *x, int64_t n, double lambda, int spherical, int max_clusters, int max_passes,
                      double clamp, int32_t *z, std::vector<double> &centres, std::vector<int64_t> &counts,
                      std::vector<double> &spread, int &K_out, int &passes_out, hipStream_t st);

struct Mlp;
hipError_t mlp_predict(const Mlp &m, const float *X, int64_t n, const uint32_t *n_dev, float *y, int grid,
                       hipStream_t s);

}  // namespace gosma

// The context behind the opaque C handle.
struct gosma_ctx {
    int device = 0;
    std::string err;

    // problems
    int n_problems = 0;
    int maxM = 0, maxN = 0;
    bool has_domain = false;
    std::vector<gosma::ProbDesc> h_prob;
    double *d_mu = nullptr, *d_isig2 = nullptr;
    float *d_w1 = nullptr, *d_pbar = nullptr;
    float4 *d_vmf = nullptr;
    gosma::ClassRange *d_cls = nullptr;
    gosma::ProbDesc *d_prob = nullptr;
    float4 *d_grec = nullptr;       // global component records for mixtures too large for LDS
    int64_t grec_stride = 0;
    std::vector<std::vector<int32_t>> gmm_order;   // original row of each sorted row, per problem

    // launch shapes of the two bound kernels (gosma_set_tiles / gosma_autotune):
    // for calls over all problems (gosma_eval_bounds) and per size bucket (the
    // search), with each bucket's problem count and largest M and N
    gosma::Tile tile11{1, 8192}, tile12{1, 8192};
    int kpieces = 1;   // pieces of the kappa interval of the S12 upper term (1, 2 or 4)
    gosma::Tile btile11[gosma::kBuckets] = {}, btile12[gosma::kBuckets] = {};
    int bucket_nprob[gosma::kBuckets] = {}, bucket_maxM[gosma::kBuckets] = {}, bucket_maxN[gosma::kBuckets] = {};

    // scratch for gosma_eval_bounds (grown on demand)
    int64_t s11_cap = 0;
    double *d_s11ub = nullptr, *d_s11lo = nullptr;
    gosma::CubeSetup *d_setup = nullptr;
    unsigned long long *d_counts = nullptr;  // work counters of timed launches (kCountSlots x kCounters)
    uint8_t *d_stage = nullptr;              // device copies of host arrays given to gosma_eval_bounds
    unsigned char *d_scratch = nullptr;      // this device's fixed scratch array (gosma_eval_bounds_noalloc)
    size_t stage_cap = 0;

    gosma::Solver *solver = nullptr;
    bool snap_ready = false;      // the solver holds the finished search of the current problems
    std::vector<uint8_t> resume;  // gosma_resume: the search state the next solve starts from
    gosma::Mlp *mlp = nullptr;
    float *rec_sink = nullptr;               // gosma_set_record_sink
    int64_t rec_cap = 0;
    unsigned long long *rec_count = nullptr;
    bool mlp_ready() const;
    std::vector<double> trace;   // 6 doubles per recorded iteration

    // kernel timing (gosma_set_timing)
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> tev;
    // record a start event if timing; returns the index to close, or -1
    int time_begin(int kind, hipStream_t s);
    void time_end(int idx, hipStream_t s);

    gosma::DevMix mix() const {
        return gosma::DevMix{d_mu,   d_isig2,  d_w1,        d_pbar,           d_vmf, d_cls,
                             d_prob, n_problems, d_grec, grec_stride, gosma::kGrecBlocks, INFINITY};
    }
};
