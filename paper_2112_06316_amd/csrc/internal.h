// Internal host-side declarations of the IFGF library.
#pragma once

#include <atomic>
#include <string>
#include <vector>

#include "../../include/ifgf.h"
#include "common.h"

namespace ifgf {

// Thrown inside the library and turned into an ifgf_status at the C ABI.
struct Error {
  ifgf_status st;
  std::string msg;
};

void hip_check(hipError_t e, const char* what);
#define HIPCHK(x) ::ifgf::hip_check((x), #x)

void set_last_error(const std::string& m);

// Device buffer owned by the plan.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  ~DevBuf();
  void alloc(size_t nbytes);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

constexpr int kNearChunk = 128;   // targets per near-field work item
constexpr int kLeafChunk = 1024;  // (cone, node) items per leaf-factor work item, rounded down to whole cones

struct LevelPlan {
  int d = 0;
  double H = 0;
  int nb = 0;                 // relevant boxes
  DevBuf start;               // int [nb + 1] point ranges (Morton order)
  DevBuf coords;              // int [nb * 3]
  DevBuf centre;              // double [nb * 3]
  DevBuf parent;              // int [nb] box index at d - 1 (d >= 2)
  DevBuf child_lo;            // int [nb + 1] children at d + 1 (d < D)
  DevBuf nbr_off, nbr;        // neighbour CSR (incl. self)
  int64_t nnbr = 0;
  DevBuf cou_off, cou;        // cousin CSR (d >= 3)
  int64_t ncou = 0;
  DevBuf pbox;                // int [n] box of each (sorted) point at this level (d >= 3)
  // cone segments (d >= 3)
  LevelGeom geom{};
  DevBuf slot;                // int [nb * ncone] relevant-cone slot or -1
  DevBuf slot_off;            // int [nb + 1]
  int nrel = 0;
  DevBuf rel_box, rel_cone;   // int [nrel]
  DevBuf Fn, Fc;              // node values (finest level only) / coefficients [nrel][P][max_rhs] complex
  DevBuf work;                // int4 [nwork]: (box, first slot, end slot, 0) chunks of this level's
  int64_t nwork = 0;          //   relevant cones, the work items of the upward pass into this level
  // cone-major upward pass into this level (IFGF_PROP_CONE): this level's
  // relevant cones sorted by (cone id, slot), in tiles of up to 8 * ti_nw
  // boxes sharing one cone id: int4 (cone id, first index into ti_slot, count, 0)
  DevBuf ti_slot, ti_tile;
  DevBuf ti_child;            // per ti_slot entry: its box's child in each octant (8 ints, -1 if none)
  DevBuf ti_geo;              // node records per (cone id of the tiles, octant), see build_ti_geo
  int64_t ntile = 0;
  // near field at the finest level: int4 [n_near] (box, first target, target
  // count, 0), boxes split into chunks of at most kNearChunk targets
  DevBuf near_work;
  int n_near = 0;
  // leaf factors at the finest level: int4 [n_leaf] (box, first item, item
  // count, 0) over the box's (relevant cone, node) items, chunks of whole
  // cones of at most kLeafChunk items
  DevBuf leaf_work;
  int n_leaf = 0;
  int ti_nw = 0;              // 0: this level uses the node formulation
  bool ti_allowed = false;    // the node-record table fits the memory rule (or CONE is forced)
  bool ti_geo_built = false;  // ti_geo holds this level's node records
  DevBuf ti_qlist;            // int [ti_nq]: the cone id of records 8 q .. 8 q + 7
  DevBuf ti_rec;              // int [nrel]: per relevant cone, the index q of its cone id's records
  int64_t ti_nq = 0;
  // Transposed upward pass into level d + 1 by gathering (built at the first
  // transposed apply, where this level has node records): the relevant cones
  // of level d + 1 in (child octant, cone id, slot) order, cut into tiles of
  // up to 64 with one (octant, cone id) bucket; per bucket, the (record,
  // group) pairs of this level's records whose nodes fall in that cone.
  DevBuf adj_tiles;           // int4 (bucket = octant * ncone(d+1) + cone id, first index into adj_slots, count, 0)
  DevBuf adj_slots;           // int [nrel(d+1)]
  DevBuf adj_gref;            // int2 (record index, group)
  DevBuf adj_gref_off;        // int [8 * ncone(d+1) + 1]
  int64_t adj_ntile = 0;
  bool adj_built = false;
  // Cousin-target pair list (one RHS): every (target, cousin box) pair of this
  // level sorted by cone slot; per pair its slot, local coordinates and centred
  // factor (plan precision), its value after the apply's first pass; per
  // target, the positions of its pairs in cousin order.
  int64_t npair = 0;
  DevBuf pr_slot;             // int [npair]
  DevBuf pr_loc;              // T4 [npair]: (ts, tt, tp, factor re)
  DevBuf pr_fim;              // T [npair]: factor im
  DevBuf pr_val;              // complex T [npair]
  DevBuf pr_off;              // int [n + 1]: target i's pairs are pr_pos[pr_off[i] .. pr_off[i + 1])
  DevBuf pr_pos;              // int [npair]
  // for the transposed apply (built on its first call): the target of each
  // sorted pair, and the runs of pairs of one slot (starts, then npair)
  DevBuf pr_tgt;              // int [npair]
  DevBuf pr_run;              // int [nrun + 1]
  int64_t nrun = 0;
  int64_t pair_rows = 0, pair_row_cones = 0;   // rows of 16 pairs, and the cone slots they meet
  // Upward-pair list of the pass d+1 -> d (sparse levels, one RHS): every
  // (node of a relevant cone of this level, child box) pair sorted by the
  // child's cone slot; per pair its slot, local coordinates in the child cone
  // and factor K(x, y_child) / K(x, y_parent) (plan precision), its value
  // after the pass's first kernel.  The pairs of node j of relevant cone s
  // are pairs up_base[s] + j * nch + t (t over the nch children of s's box,
  // in child order) before sorting; up_pos maps them to sorted positions.
  int64_t nup = 0;
  bool up_use = false;        // the pass d+1 -> d runs from this list
  DevBuf up_slot;             // int [nup]
  DevBuf up_loc;              // T4 [nup]: (ts, tt, tp, factor re)
  DevBuf up_fim;              // T [nup]: factor im
  DevBuf up_val;              // complex T [nup]
  DevBuf up_base;             // int [nrel + 1]
  DevBuf up_pos;              // int [nup]
  // for the transposed apply (built on its first call): the parent node
  // (s * P + j) of each sorted pair, and the runs of pairs of one slot
  DevBuf up_node;             // int [nup]
  DevBuf up_run;              // int [up_nrun + 1]
  int64_t up_nrun = 0;
  // statistics
  int64_t cousin_pairs = 0;
  int64_t prop_evals = 0;     // child interpolations into level d-1 nodes
};

}  // namespace ifgf

struct ifgf_plan_s {
  int64_t n = 0;
  int D = 0;
  int64_t n_src = 0;          // points carrying densities (caller indices < n_src); the rest are targets only
  bool pairs = false;         // every level 3..D holds its cousin-target pair list
  bool adj_pairs = false;     // ... and its transposed-apply index (pr_tgt, pr_run)
  bool pairs_rg = false;      // ... with room for 16 values per pair (RHS groups of 16)
  std::atomic<int> batch_refs{0};   // batches built over this plan (their queues point into its buffers)
  ifgf::DevBuf uext;          // plans with targets: the apply's result at every point, caller's order
  double k = 0, eta = 0;
  ifgf_options opt{};
  int P = 0;                  // p_s * p_ang^2
  double L = 0, corner[3] = {0, 0, 0};
  ChebTab cheb{};
  // Chebyshev node-value -> coefficient matrices (row-major n x n)
  ifgf::DevBuf Ms, Ma;        // double
  ifgf::DevBuf Msf, Maf;      // float
  ifgf::DevBuf perm;          // int [n]: Morton position -> caller index
  ifgf::DevBuf keys;          // uint32 [n]
  ifgf::DevBuf pts, nrm, w;   // sorted geometry (double)
  ifgf::LevelPlan lev[IFGF_MAX_LEVELS];
  ifgf::DevBuf a;             // gathered coefficients w * sigma, [n][max_rhs] complex (plan precision)
  ifgf::DevBuf uacc;          // near-field results, [n][max_rhs] complex (plan precision)
  ifgf::DevBuf tpart;         // cousin-target level sums, [D - 2][n] complex (plan precision)
  ifgf::DevBuf adj_g[IFGF_MAX_LEVELS];   // transposed-apply coefficient-space buffers
  ifgf::DevBuf err;           // int [4] device error flags
  int64_t near_pairs = 0;
  // kernel timing (ifgf_plan_set_profiling)
  std::vector<hipEvent_t> ev;        // 2 per timed launch
  std::vector<int> ev_stage;
  int ev_used = 0;
  std::atomic<int> busy{0};
  int last_rhs = 0;
};

namespace ifgf {

// One segment of the batch work queue: items [first, first + count) of one
// kind, geometry and level.  Before an item, wait until ctr[dep0] >= need0 and
// ctr[dep1] >= need1 (dep < 0: none); after it, increment ctr[done].
struct BSeg {
  int type, geom, level, count;
  int first;
  int dep0, need0, dep1, need1;
  int done;
};

}  // namespace ifgf

struct ifgf_batch_s {
  std::vector<ifgf_plan_s*> plans;   // not owned
  ifgf::DevBuf segs;                 // BSeg [nseg]
  ifgf::DevBuf seg_of;               // int [total]: segment of each queue item
  ifgf::DevBuf geoms;                // per-geometry device descriptors
  ifgf::DevBuf ctr;                  // int [nctr]: queue head, then 16 completion counters per geometry
  ifgf::DevBuf err;                  // int [4]: bit 0 = a dependency wait hit the poll limit
  int nseg = 0, total = 0, nctr = 0;
  int grid = 0, block = 0;
  size_t smem = 0;
  int spin_limit = 1 << 22;
  int device = 0;                    // current device when the batch was created
  std::atomic<int> busy{0};
};

namespace ifgf {

// primitives.hip
void scan_exclusive_u8(const uint8_t* in, int* out, int64_t n, hipStream_t s);   // out[n] = total
void scan_exclusive_i32(const int* in, int* out, int64_t n, hipStream_t s);      // out[n] = total
int64_t sort_padded_length(int64_t n);                                              // capacity sort_u64 needs
void sort_u64(uint64_t* data, int64_t n, hipStream_t s);                          // ascending, in place

// plan.hip
void build_plan(ifgf_plan_s* p, const double* pts, const double* nrm, const double* w, hipStream_t s);
// (Re)build the cone-major tiles of the upward pass into level d with tiles of
// 8 * nw_req boxes (nw_req < 0: heuristic; 0: node formulation); returns nw.
int build_cone_tiles(ifgf_plan_s* p, int d, int nw_req, hipStream_t s);

// apply.hip
void run_apply(ifgf_plan_s* p, const void* sigma, void* u, int nrhs, int dtype, int stage_mask,
               int level_lo, int level_hi, hipStream_t s);
void run_adjoint(ifgf_plan_s* p, const void* v, void* out, int nrhs, int dtype, int conj, hipStream_t s);
void run_export_nodes(ifgf_plan_s* p, void* dst, hipStream_t s);   // finest level's node values, device dst
void run_far_field(ifgf_plan_s* p, const void* sigma, int64_t ndir, const double* dirs, void* uinf, int dtype,
                   hipStream_t s);
void run_autotune(ifgf_plan_s* p, int reps, ifgf_tune_report* rep, hipStream_t s);
// Builds the cousin-target pair lists (plan time) where the order, precision
// and size allow; sets p->pairs.
void build_target_pairs(ifgf_plan_s* p, hipStream_t s);
void release_target_pairs(ifgf_plan_s* p);
// upward pair lists of the pass d+1 -> d (sparse levels)
bool up_pairs_possible(const ifgf_plan_s* p, int d);
void build_up_pairs(ifgf_plan_s* p, int d, hipStream_t s);
void release_up_pairs(LevelPlan& lv);
void build_plan_up_pairs(ifgf_plan_s* p, hipStream_t s);

// solve.hip: restarted GMRES on (alpha I + A) sigma = f (complex128 device vectors).
void run_gmres(ifgf_plan_s* p, const void* f, void* sigma, const ifgf_gmres_options& o, int32_t* iters,
               double* rel_res, double* history, hipStream_t s);

void run_batch_prepare(ifgf_batch_s* b);
// ctr: the launch's completion counters (b->nctr ints); nullptr = the batch's own buffer.
void run_batch_apply(ifgf_batch_s* b, const void* const* sigma, void* const* u, int dtype, int* ctr, hipStream_t s);
// Device address of the fixed counter array (BATCH_STATIC_COUNTERS ints) on `device`,
// which must be the current device; looked up once per device.
constexpr int BATCH_STATIC_COUNTERS = IFGF_BATCH_NOALLOC_COUNTERS;
constexpr int kBatchCtrPerGeom = 32;   // completion counters per geometry of a ragged batch
static_assert(BATCH_STATIC_COUNTERS == 1 + kBatchCtrPerGeom * IFGF_BATCH_MAX, "noalloc counter array");
int* batch_static_counters(int device);

// The cone-major tiles' node records of level d (one per cone id in qlist and
// octant), computed on the GPU into p->lev[d].ti_geo.
void build_ti_geo(ifgf_plan_s* p, int d, const std::vector<int>& qlist, hipStream_t s);
size_t ti_geo_bytes(int ps, int pa, bool f32);   // one (cone id, octant) record
bool supported_order(int ps, int pa, int precision);   // compiled in for this precision
int prop_chunk(int P);
bool cone_prop_supported(const ifgf_plan_s* p);

// Brackets one kernel launch with events when profiling is enabled.
struct StageTimer {
  ifgf_plan_s* p;
  hipStream_t s;
  int slot = -1;
  StageTimer(ifgf_plan_s* pp, hipStream_t ss, int stage);
  ~StageTimer();
};

}  // namespace ifgf
