// Internal declarations shared by the host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sg.h"

namespace sgk {

constexpr int kMaxCheb = 16;     // largest supported Chebyshev degree
constexpr int kMaxLevels = 16;   // largest supported chaos degree + 1
constexpr int kPcgPartials = 7;  // per-tile partial-sum arrays of the inner solver
constexpr int kRedBlocks = 1024; // blocks of the FP64 reduction kernels

// Tiles of the inner PCG on an nx x nx grid. tile == 16: square 16 x 16 tiles.
// Otherwise banded tiles of `rows` node rows whose 64-column regions hold the
// tile plus its Chebyshev halo (degree - 1 nodes, at least one) plus one more
// node on each side that is not the grid's edge (band_ntx below). Tiles are
// numbered row-major: tile t is column (t % ntx) of tiles and band row t / ntx.
// Band heights: a taller band recomputes less of the halo. Bands are 128 rows
// high in FP64 and 256 in FP32 (one band row at 256^2), worked by one group of
// 16 waves per block without the next-tile prefetch, so that a wave's rows fit
// its registers; launches with few tiles may take shorter bands (64 rows,
// with the prefetch, or in FP32 128 rows; pcg_band_rows).
template <typename T>
constexpr int kBandRowsOf = sizeof(T) == 4 ? 256 : 128;
// Highest Chebyshev degree served by banded tiles: the halo (degree - 1) plus
// one node on each side leaves 32 interior columns of 64 lanes at degree 16.
// Higher degrees take 16 x 16 tiles.
constexpr int kBandMaxDegree = 16;
// Band heights of launches with few tiles: shorter bands give more tiles, so a
// launch of a few columns still spreads over the compute units. FP32 also has
// the FP64 default height between its own and the shortest.
constexpr int kBandRowsSmall = 64;
constexpr int kBandRowsMid = 128;
inline int band_rows(int inner_precision, int) {
  return inner_precision == 32 ? kBandRowsOf<float> : kBandRowsOf<double>;
}
// Column widths of banded inner tiles: a tile's region is one wavefront (64
// grid columns) wide and needs a halo of h = (degree - 1) + 1 columns (the
// Chebyshev halo plus one node for q = K_0 p and for the residual of a warm
// start; at least 2) on each side that is not the grid's edge. Inner tiles
// have 64 - 2h interior columns; the first and the last tile of a band row
// have their regions end at the grid's edge and take 64 - h; a grid at most
// 64 columns wide is one tile.
__host__ __device__ inline int band_halo(int degree) { return (degree - 1 > 1 ? degree - 1 : 1) + 1; }
// Tiles across a grid row for regions of 64 columns with a halo of h columns.
__host__ __device__ inline int band_cols(int nx, int h) {
  const int a = 64 - h, w = 64 - 2 * h;
  if (nx <= 64) return 1;
  return 2 + (nx > 2 * a ? (nx - 2 * a + w - 1) / w : 0);
}
__host__ __device__ inline int band_ntx(int nx, int degree) { return band_cols(nx, band_halo(degree)); }

inline void pcg_tiling(int nx, int degree, int tile, int rows, int& ntx, int& ntiles) {
  if (tile == 16) {
    ntx = (nx + 15) / 16;
    ntiles = ntx * ntx;
    return;
  }
  ntx = band_ntx(nx, degree);
  ntiles = ntx * ((nx + rows - 1) / rows);
}
// Tiles of the busiest block when nwork banded tiles (one 16-wave group per
// block) take the inner solver's automatic grid on ncu compute units: one tile
// per block when they fit, else two per block on at most ncu blocks, the
// tiles split evenly over the grid (shares differ by at most one).
inline long pcg_busiest_block(long nwork, long ncu) {
  if (nwork <= ncu) return 1;
  const long grid = (nwork + 1) / 2 < ncu ? (nwork + 1) / 2 : ncu;
  return (nwork + grid - 1) / grid;
}
// Band height of a banded inner launch of ncols columns with automatic tiles.
// A launch with fewer tiles of the precision's default height than compute
// units may take shorter bands, which spread it over more of them; but a block
// that then works two short tiles per phase sweeps more rows than one tall
// one. The height taken is the one whose busiest block sweeps the fewest
// region rows (band rows plus the halo above and below) per iteration, the
// shorter on a tie; FP32 has the FP64 default height as a middle one.
inline int pcg_band_rows(int nx, int degree, int inner_precision, int ncols, int ncu) {
  const int def = band_rows(inner_precision, degree);
  const long ntx = band_ntx(nx, degree);
  auto tiles = [&](int rows) { return (long)ncols * ntx * ((nx + rows - 1) / rows); };
  if (tiles(def) >= ncu) return def;
  const int halo = 2 * band_halo(degree);
  int best_rows = def;
  long best = pcg_busiest_block(tiles(def), ncu) * (def + halo);
  const int shorter[2] = {inner_precision == 32 ? kBandRowsMid : 0, kBandRowsSmall};
  for (int rows : shorter) {
    if (rows <= 0 || rows >= best_rows) continue;
    const long cost = pcg_busiest_block(tiles(rows), ncu) * (rows + halo);
    if (cost <= best) {
      best = cost;
      best_rows = rows;
    }
  }
  return best_rows;
}

// Chaos neighbour lists of the Hermite Galerkin matrices G_k (k >= 1): for
// each chaos row a, the entries (k, b, g) with (G_k)_{ab} = g != 0 split into
// lower neighbours (b = a - e_k, g = sqrt(a_k)) and upper neighbours
// (b = a + e_k, g = sqrt(a_k + 1)). CSR over rows; an entry is packed as
// b | (k << 20) with k in 1..M.
template <typename T>
struct ChaosLists {
  const int* lo_ptr;
  const int* lo_ent;
  const T* lo_g;
  const int* up_ptr;
  const int* up_ent;
  const T* up_g;
};

// out[a] = rcoef * rsrc[a] + diag * K_Lap in[a] + sgn * sum_{entries (k,b,g) of a} g * K_k in[b]
// for chaos rows a in [row0, row0 + nrows). Columns live at base + col * n.
template <typename T>
struct SgOpArgs {
  int n_e;
  int nx;
  long n;
  int row0;
  int nrows;
  int use_lower;
  int use_upper;
  T diag;
  T rcoef;
  T sgn;
  const T* in;
  const T* rsrc;
  T* out;
  const T* a;  // [M][n_e * n_e] element coefficients of K_1..K_M
  ChaosLists<T> lists;
  const int* active;  // if not null: the launch does nothing while *active == 0
};

// Dense per-row neighbour tables [P][M] for the strip kernel: lo[a*M + k] is the
// row index of a - e_{k+1} (or -1) with coefficient glo = sqrt(a_{k+1}); up the same
// for a + e_{k+1} with gup = sqrt(a_{k+1} + 1).
template <typename T>
struct StripTables {
  const int* lo;
  const int* up;
  const T* glo;
  const T* gup;
  int M;
  int blocks_per_band;  // row chunks per grid band (0 = default)
  // Compact per-row entry lists for the occupancy variant: entries of row a are
  // ent_ptr[a] .. ent_ptr[a+1]-1, each (k, lo, up) with glo/gup (absent side: index a, weight 0).
  const int* ent_ptr;
  const int* ent_k;
  const int* ent_lo;
  const int* ent_up;
  const T* ent_glo;
  const T* ent_gup;
  int variant;  // 0: coefficients in registers, 1: coefficients loaded per entry
};

// Row groups of one use of the SG operator (the full matvec, or one coupling
// product) for the y-marching kernel. Group g owns rows grows[gptr[g] ..
// gptr[g+1]-1]. A group of kind 0 holds at most kMarchRGU rows that have upper
// neighbours (all KL terms used, neighbours from the dense [P][M] tables); a
// group of kind 1 holds at most kMarchRGL rows with lower neighbours only,
// whose KL terms are gathered into kMarchNS slots: lk[g][s] is the KL term
// (0-based, -1 unused) of slot s and lcol/lw[g][j][s] the lower neighbour of
// row j through that term (-1 none) and its weight. The grid rows 1..nx are cut
// into nseg segments of seg_rows node rows; a block handles one (segment,
// group) pair.
constexpr int kMarchRGU = 2;
constexpr int kMarchRGL = 6;
constexpr int kMarchNS = 4;
// Spatial pieces of the piece kernel: W interior node columns per piece (one
// wavefront holds W + 2 columns with the halo), nstrips = ceil(nx / W) pieces
// across, TY node rows per piece, nyseg = ceil(nx / TY) pieces up. W = 0: the
// piece kernel is not used. max_waves_per_cu caps the resident waves (0: as
// many as fit).
struct PieceGeom {
  int W;
  int nstrips;
  int TY;
  int nyseg;
  int max_waves_per_cu;
};
struct MarchJob {
  const int* gptr;
  const int* grows;
  const int* gkind;
  const int* lk;
  const int* lcol;
  const double* lw;
  int ngroups;
  int nseg;
  int seg_rows;
  PieceGeom piece;
};

template <typename T>
void launch_sgop(const SgOpArgs<T>& args, const StripTables<T>& tab, const MarchJob* job, hipStream_t s);

// Row-staged SG operator (the full FP64 operator Y = sum_k K_k U G_k^T): a block
// of kStageWaves waves stages node rows of all P chaos columns, for a segment of
// 32 node columns (30 outputs plus a halo node on each side), in LDS; every half
// wave (32 lanes) accumulates one output column's element sums from the staged
// rows, term by term. The mean term of an output (its own column, coefficient
// theta0) is handled by its slot; the slot's term list holds the Galerkin
// neighbours. A slot pairs two outputs (one per half) whose neighbour weights
// are equal in order, so a term's weight is one value for both halves; the
// input column and the KL row differ per half. The term and slot tables are
// copied into LDS at the start of the kernel.
constexpr int kStageWaves = 16;
constexpr int kStageLanes = 32;            // node columns per staged segment (lanes of a half wave)
constexpr int kStageOut = kStageLanes - 2; // output node columns per segment
constexpr int kStageSlots = 10;            // output pairs per wave
constexpr int kStagePre = 9;               // staged values per thread and row: P * 32 <= 9 * 1024
struct StageTerm {       // 16 bytes
  unsigned short b[2];   // per half: input column
  unsigned char k[2];    // per half: KL index (1..M)
  unsigned short pad;
  double g;              // Galerkin weight of the term for both halves
};
struct StageSlot {       // 8 bytes
  unsigned short out[2]; // output chaos index per half (0xFFFF: none)
  unsigned short t0, nt; // first term and term count
};
struct StageJob {
  const StageTerm* terms;
  const StageSlot* slots;
  const int* wslot;  // [kStageWaves + 1]: slot range of each wave
  int P, M;
  int nterms, nslots;
  int TY;            // output node rows per piece
  int nseg, nyseg;   // pieces: nseg segments by nyseg row bands
};
// LDS bytes of the row-staged kernel, 0 if the problem does not fit it.
size_t stage_lds_bytes(int P, int M, int nterms, int nslots);
void launch_stage(const SgOpArgs<double>& args, const StageJob& job, hipStream_t s);

// Largest number of KL terms served by the piece kernel (dense [P][M] tables).
constexpr int kPieceMaxM = 12;

// Resident blocks per CU of the y-marching kernel for this M and block size (0 if unsupported).
int march_blocks_per_cu(int M, int block);
bool march_supported(int n_e, int M);

// Persistent batched PCG on K_0 = theta0 * K_Lap (one independent solve per column).
struct PcgScratch {
  double* part;        // [kPcgPartials][ncols][ntiles] per-tile partial sums
  unsigned* arrivals;  // [ncols] monotonic per-column arrival counters
  int* iters;          // [ncols]
  int* status;         // [1] nonzero if a bounded wait expired
};

template <typename T>
struct PcgArgs {
  int nx;
  long n;
  int ncols;
  const T* B;
  T* X;
  T* R0;
  T* R1;
  T* P0;
  T* P1;
  T* Q;
  T* Z;
  PcgScratch sc;
  int ntx;
  int ntiles;
  int rows;    // band height of banded tiles (as in the tiling of ntx, ntiles)
  int degree;
  int maxit;
  double rtol;
  int warm;    // start each column from the contents of its x (banded tiles), else from 0
  long per_block;  // work items (tiles) per block; 0 = the work list split evenly over the grid
  int no_coop;     // 1: an ordinary launch (graph capture) instead of a cooperative one
  T c0;        // centre weight of K_0: theta0 * 8/3
  T c1;        // neighbour weight of K_0: -theta0 / 3
  T inv_diag;  // 1 / (theta0 * 8/3)
  T inv_theta; // 1 / centre of the Chebyshev interval
  T w8;        // 1/8: neighbour weight of the Jacobi-scaled stencil D^-1 K_0 (a runtime value, so
               // that the kernels take it from a scalar register)
  T chebA[kMaxCheb];
  T chebB[kMaxCheb];
};

// Per-problem constants of a ragged launch (same meaning as the fields of PcgArgs).
template <typename T>
struct PcgConsts {
  T c0, c1, inv_diag, inv_theta, w8;
  T chebA[kMaxCheb];
  T chebB[kMaxCheb];
};

// A ragged column set: columns from several problems with their own grids.
// Column c has nx[c] nodes per side, ntx[c] tiles per side, ntiles[c] tiles
// whose work indices start at tbase[c] (prefix sums, nwork in total), belongs
// to problem prob[c] (constants consts[prob], skipped while active[prob] == 0)
// and keeps its PCG state in the n-vectors b, x, r0, r1, p0, p1, q, z.
template <typename T>
struct PcgCols {
  const int* nx;
  const int* ntx;
  const int* ntiles;
  const long* tbase;
  const int* prob;
  const T* const* b;
  T* const* x;
  T* const* r0;
  T* const* r1;
  T* const* p0;
  T* const* p1;
  T* const* q;
  T* const* z;
  const PcgConsts<T>* consts;
  const int* active;
  long nwork;
  // Optional compaction: if act is not null, the launch covers only the
  // columns act[0 .. *nact - 1] (indices into the arrays above, in order);
  // their per-tile partials start at cbase[i] (prefix sums over the listed
  // columns, *nwork_act in total). Scratch arrays are indexed by list position.
  const int* act;
  const int* nact;
  const long* cbase;
  const long* nwork_act;
};

template <typename T>
hipError_t launch_pcg(const PcgArgs<T>& args, int tile, int max_blocks, hipStream_t s);

// Ragged launch over `ncols` columns described by `cols`; degree, maxit, rtol and
// the scratch come from `args`. A regular launch whose grid fits on the device
// at once (so it can be captured into a graph); every wait is bounded.
template <typename T>
hipError_t launch_pcg_ragged(const PcgArgs<T>& args, const PcgCols<T>& cols, int tile, int max_blocks, hipStream_t s);

template <typename T>
size_t pcg_scratch_bytes(int ncols, int ntiles);

// FP64 BLAS-1 style kernels with deterministic two-stage reductions.
void launch_dots(const double* const* a, const double* const* b, int ndots, long N, double* partials,
                 double* out, hipStream_t s);
void launch_fcg_update(double* x, double* r, const double* p, const double* q, double alpha, long N,
                       double* partials, double* out, hipStream_t s);
void launch_xpby(double* p, const double* z, double beta, long N, hipStream_t s);
void launch_axpby(double* y, const double* x, double a, double b, long N, hipStream_t s);  // y = a x + b y
void launch_fill(double* y, double v, long N, hipStream_t s);
void launch_copy_d2f(float* dst, const double* src, long N, hipStream_t s);
void launch_copy_f2d(double* dst, const float* src, long N, hipStream_t s);
void launch_copy_d2d(double* dst, const double* src, long N, hipStream_t s);
void launch_sub(double* r, const double* f, const double* y, long N, hipStream_t s);  // r = f - y

// Adjoint support.
void launch_qoi(const double* U, const double* wm, const double* wv, long n, int P, double* partials,
                double* out, hipStream_t s);
void launch_qoi_grad(const double* U, const double* wm, const double* wv, long n, int P, double* G,
                     hipStream_t s);
struct ContractArgs {
  int n_e;
  int nx;
  long n;
  int M;
  int P;
  const double* Lam;
  const double* U;
  const double* c;      // [M][n_e * n_e] sigma * phi_k(e)
  const int* pair_ptr;  // [M + 1] start of the (a, b, g) pairs of G_k, k = 1..M
  const int* pair_a;
  const int* pair_b;
  const double* pair_g;
  double* partials;     // [nblocks][M + 1]
  double* out;          // [M + 1]
};
void launch_contract(const ContractArgs& args, hipStream_t s);

// ---- multi-problem batch: the flexible CG of many independent problems with
// its scalars on the device, so that one outer iteration of the whole batch is
// a fixed sequence of launches (it can be captured into a graph).
constexpr int kBatchBlocks = 256;  // blocks per problem of the batched vector kernels

struct BatchScal {
  double fn2;        // ||f||^2
  double rr;         // ||r||^2 after the last update
  double pq, pr, zq;
  double pq_prev;
  double rtol2;      // the solve stops once rr <= rtol2 (= rtol^2 ||f||^2)
  int it;            // outer iterations done
  int status;        // SG_NOT_CONVERGED while iterating, then SG_OK or SG_BREAKDOWN
  long long inner_it;  // inner PCG iterations summed over the solve
};

// Per problem b: the length N[b] = n P of its blocks and their addresses.
struct BatchVecs {
  int nprob;
  const long* N;
  double* const* x;
  const double* const* f;
  double* const* r;
  double* const* z;
  double* const* p;
  double* const* q;
  void* const* rw;  // residual in inner precision
  void* const* zw;  // preconditioned residual in FP32 (FP32 inner only)
  BatchScal* sc;
  int* active;      // 1 while problem b iterates; every batched launch skips it otherwise
  double* part;     // [nprob][kBatchBlocks][2]
  long maxN;
};

void launch_batch_init(const BatchVecs& V, double rtol, hipStream_t s);
void launch_batch_dot_zq(const BatchVecs& V, hipStream_t s);
void launch_batch_dirupdate(const BatchVecs& V, hipStream_t s);   // p = z + beta p, beta = -zq / pq_prev
void launch_batch_dot_pq_pr(const BatchVecs& V, hipStream_t s);
void launch_batch_update(const BatchVecs& V, hipStream_t s);      // alpha = pr / pq; x += alpha p, r -= alpha q; test
template <typename T>
void launch_batch_to_inner(const BatchVecs& V, hipStream_t s);    // rw = r
void launch_batch_from_inner(const BatchVecs& V, hipStream_t s);  // z = zw
void launch_batch_count_iters(const int* iters, const int* act, const int* nact, const int* prob, int ncols,
                              BatchScal* sc, const int* pcg_status, int* sticky_status, hipStream_t s);
// List of the columns of a ragged set whose problem is still active and has
// chaos degree pdeg >= pmin, with the prefix sums of their tile counts (the
// partial slots of the next launch).
void launch_batch_compact(const int* prob, const int* ntiles, int ncols, const int* active, const int* pdeg, int pmin,
                          int* act, int* nact, long* cbase, long* nwork_act, hipStream_t s);

}  // namespace sgk

// Host-side context behind sg_handle.
struct sg_ctx {
  int n_e, M, p, P, nx;
  int family;  // SG_FAMILY_*
  long n;
  double theta0, sigma;
  double lmin, lmax;  // spectrum of D^-1 K_0
  std::vector<double> s;
  std::vector<int> off;
  std::vector<int> alpha;  // [P][M]
  sg_opts opts;
  hipStream_t stream;
  int num_cu;
  int tile;
  int mv_blocks_per_band;
  int mv_variant;  // 0, 1: band kernels; 2: y-marching kernel
  int pcg_max_blocks;
  bool march_ok;
  int mv_seg_per_xcd = 0;  // grid segments per XCD of the y-marching kernel (0 = automatic)
  int mv_piece_rows = 0;   // node rows per piece of the piece kernel (0 = default 16)
  int mv_piece_waves = 0;  // cap on resident waves per CU of the piece kernel (0 = as many as fit)
  // row-staged kernel for the full operator (sg_matvec and the outer CG products)
  bool stage_ok = false;   // tables built and the sizes fit
  int mv_stage = 0;        // node rows per piece when the full operator uses it, 0 = off
  sgk::StageJob stage{};
  std::vector<sgk::MarchJob> mjobs;
  std::vector<int> st_lo_h, st_up_h;  // host copies of the dense neighbour tables (row groups)
  std::vector<double> st_glo_h;
  int *mj_ptr_d, *mj_rows_d, *mj_kind_d, *mj_lk_d, *mj_lcol_d;
  double* mj_lw_d;
  const int* mask = nullptr;  // device flag of a batch member: SG operator launches skip while it is 0
  // host copies of the chaos lists (for counters)
  std::vector<int> lo_ptr, up_ptr;
  // device arrays inside the workspace
  char* ws;
  size_t ws_bytes;
  double* a64;
  float* a32;
  double* c64;
  int *lo_ptr_d, *lo_ent_d, *up_ptr_d, *up_ent_d;
  double *lo_g64, *up_g64;
  float *lo_g32, *up_g32;
  int *st_lo_d, *st_up_d;
  int *en_ptr_d, *en_k_d, *en_lo_d, *en_up_d;
  double *en_glo64, *en_gup64;
  float *en_glo32, *en_gup32;
  double *st_glo64, *st_gup64;
  float *st_glo32, *st_gup32;
  int *pair_ptr_d, *pair_a_d, *pair_b_d;
  double* pair_g_d;
  double *r, *z, *pv, *q, *lam, *tmp, *rhs;  // FP64 n x P blocks
  void* rw;  // inner-precision working residual, n x P
  void* zw;  // inner-precision output, n x P (FP32 only)
  void *pR0, *pR1, *pP0, *pP1, *pQ, *pZ;  // inner PCG state, n x maxcols
  int pcg_maxcols;
  sgk::PcgScratch pcgsc;
  double* red_part;  // reduction partials
  double* red_out;   // reduction results (device)
  std::vector<double> host_out;  // host mirror of red_out
  long inner_it_acc;
  double inner_ms_acc;
  double inner_bytes_acc;
  long inner_launch_acc;
  hipEvent_t ev0, ev1;
  int inner_it_max[sgk::kMaxLevels];
  // Inner launches whose iteration counts, status word and timing are read
  // back later (once per preconditioner action instead of once per launch):
  // each has a pair of events from evpool and a slice of the pinned host
  // buffer iters_host (its column counts), status_host[i] its status word.
  struct PendingLaunch {
    int ncols, level, tile, warm, wsize;
    long slot;
    bool timed;  // its events were recorded (not inside a graph capture)
  };
  static constexpr int kMaxPending = 64;
  std::vector<PendingLaunch> pending;
  hipEvent_t evpool[2 * kMaxPending];
  int nev = 0;             // events created in evpool
  int* iters_host = nullptr;   // pinned, iters_cap ints
  int* status_host = nullptr;  // pinned, kMaxPending ints
  long iters_cap = 0, iters_used = 0;
  // one preconditioner action captured into a HIP graph (opts.use_graph)
  bool capturing = false;   // inner launches are ordinary launches and never settle the read-back
  hipGraph_t pc_graph = nullptr;
  hipGraphExec_t pc_exec = nullptr;
  int pc_kind = -1;                      // preconditioner of the captured action
  const double* pc_R = nullptr;          // its input and output blocks
  double* pc_Z = nullptr;
  std::vector<PendingLaunch> pc_pending; // the read-back records of one replay
  long pc_iters_used = 0;
  long pc_nbmv = 0, pc_nbs = 0;          // block products and solves of one action
  int defer = 0;           // > 0: run_pcg leaves the read-back to flush_inner
  void* static_scratch = nullptr;  // this device's static scratch array (sg_inner_solve_static)
};
