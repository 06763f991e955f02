// C ABI of the gfx950 FE-LBM step (declared in include/felbm.h): context and
// device memory management, mesh upload, the per-step launch sequence and
// the read-back / checkpoint / timing entry points.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adjoint.hpp"
#include "felbm.h"
#include "kernels.hpp"
#include "mesh_prep.hpp"

using namespace felbm;

namespace {

enum KernelId {
  K_MOMENTS = 0, K_REDUCE, K_GRAD, K_EFLUX, K_LAPC, K_GRADMU, K_LAPMU, K_NODEF, K_RHS, K_SWEEP_FIRST, K_SWEEP_MID,
  K_SWEEP_LAST, K_ADJ_PREP, K_ADJ_FORCE, K_ADJ_STREAM, K_ADJ_GMU, K_ADJ_MU, K_ADJ_GC, K_ADJ_NODE, K_RESID,
  K_LAPC_OP, K_LAPMU_OP, K_COUNT
};
const char* const kKernelNames[K_COUNT] = {"moments_collide", "reduce_final", "elem_grad", "edge_flux", "lapC_mu",
                                           "elem_gradmu", "elem_lapmu", "node_forces", "rhs_gather", "sweep_first",
                                           "sweep_mid", "sweep_last", "adj_prep", "adj_force", "adj_stream",
                                           "adj_gmu", "adj_mu", "adj_gC", "adj_node", "residual",
                                           "lapC_mu_op", "lapmu_op"};

struct KStat {
  int64_t launches = 0;
  double total_ms = 0.0;
  double bytes = 0.0;
};

struct PendingTiming {
  int kid;
  hipEvent_t start, stop;
};

constexpr uint32_t kStateMagic = 0x4645424du;  // "FEBM"

struct StateHeader {
  uint32_t magic;
  int32_t precision;
  int64_t n_nodes;
  int64_t step;
  int64_t payload_bytes;
  uint64_t perm_hash;  // internal node order the payload is laid out in
};

inline int grid_for(int64_t n) {
  int64_t b = (n + BLOCK - 1) / BLOCK;
  b = (b + 7) / 8 * 8;  // multiple of 8 for the XCD remap
  return (int)std::max<int64_t>(b, 8);
}

// Scratch of felbm_diagnostics_noalloc, which allocates nothing: the FP64
// block partials of the reductions ([NRED][blocks], row stride the launch's
// block count), then the reduced record and the non-finite flag.  Blocks of
// 256 nodes, at most kNoAllocMaxBlocks of them: meshes of up to 8,388,608
// nodes; 1.5 MiB per device, held until the process ends.  Every context on
// a device shares that device's copy.
constexpr int kNoAllocMaxBlocks = 32768;
constexpr size_t kNoAllocRecordOffset = (size_t)NRED * kNoAllocMaxBlocks;  // in doubles
constexpr size_t kNoAllocDoubles = kNoAllocRecordOffset + 16;              // record (56 B) + flag
static_assert(sizeof(DiagRecord) + sizeof(int32_t) <= 16 * sizeof(double), "noalloc record slot");

// Per-device address of `scratch`, taken once per device with that device
// current (the array's name is only a host-side stand-in for it).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

// Called by felbm_create with the context's device current.
int noalloc_scratch_for_current_device(int device, void** out, std::string& err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "create: device index beyond the no-alloc scratch table";
    return FELBM_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("create: hipGetSymbolAddress of the no-alloc scratch failed: ") + hipGetErrorString(e);
      return FELBM_EDEVICE;
    }
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return FELBM_OK;
}

}  // namespace

struct felbm_ctx {
  felbm_params prm{};
  StepParams sp{};
  std::string err;
  int device = 0;
  hipStream_t own_stream = nullptr, stream = nullptr;
  bool has_mesh = false, has_state = false;
  int64_t N = 0, Np = 0, E = 0, W = 0, offdiag_nnz = 0, sell_entries = 0;
  size_t rs = 8;
  int64_t step = 0;
  Band band{};
  std::vector<double> cheb_w;  // Richardson step lengths (reciprocal Chebyshev roots), in sweep order
  // mesh (device)
  int32_t *tri = nullptr, *enbr = nullptr, *n2e_ptr = nullptr, *n2e = nullptr, *wall_nbr = nullptr;
  int32_t *sell_ptr = nullptr, *sell_col = nullptr;
  double *geo = nullptr, *wall_len = nullptr, *bc = nullptr, *mass = nullptr, *xy = nullptr;
  double *pvol = nullptr, *eflux = nullptr;  // patch volume per node; edge fluxes [3][E]
  void* Fn = nullptr;                         // nodal forces [18][Np] (nodal force scheme)
  double* lapmu_n = nullptr;                  // nodal lap mu [N] (collision-step nodal scheme)
  void *geor = nullptr, *sell_val = nullptr;
  uint8_t* is_wall = nullptr;
  // state and work buffers (device)
  void *pop = nullptr, *f = nullptr, *xa = nullptr, *xb = nullptr;
  double *Cn = nullptr, *mu = nullptr, *lapC = nullptr, *gC = nullptr, *gmu = nullptr, *lapmu = nullptr;
  void *pn = nullptr, *uxn = nullptr, *uyn = nullptr, *gp = nullptr;
  // precomputed operators of the chemical-potential chain (see k_lapC_mu_op, k_lapmu_op)
  int32_t *lop_ptr = nullptr, *lop_col = nullptr, *wptr = nullptr, *eopp = nullptr;
  int2* wab = nullptr;
  double* wlen = nullptr;
  void *lop_w = nullptr, *ew = nullptr;
  // LDS-tiled solve: per-tile halo lists and matrix rows with local slots
  bool use_lds = false;
  int ntiles = 0, tile_slots = 0;
  int32_t *tile_off = nullptr, *halo_off = nullptr, *halo = nullptr;
  uint16_t* tslot = nullptr;
  void* tval = nullptr;
  // LDS-tiled right-hand side (FP32): per-tile incident-element entries with vertex slots
  bool use_rhs_lds = false;
  int32_t* rhs_off = nullptr;
  int2* rhs_ent = nullptr;
  double* gaos = nullptr;  // element geometry records [E][4]
  // adjoint: element reverse adjacency, caller<->internal maps, reverse buffers, checkpoints
  int32_t *erev = nullptr, *d_node_perm = nullptr;
  void *lam = nullptr, *lhat = nullptr;
  double *ea = nullptr, *lgmu = nullptr, *lgC = nullptr, *lmu = nullptr, *gomega = nullptr;
  void* lqe = nullptr;  // lam_q per element [18][E], compute precision
  void* ck_buf = nullptr;     // checkpoints every ck_every steps
  void* seg_buf = nullptr;    // replayed states of one segment
  int64_t ck_steps = 0, ck_every = 0, ck_count = 0, ck_start = 0;
  int64_t ck_run = 0, ck_next_run = 0;  // identifier of the run the checkpoints belong to (0 = none)
  // sampled solver residual
  int64_t residual_every = 0, residual_step = -1;
  void* noalloc_scratch = nullptr;  // this device's address of the no-alloc scratch array
  double* res_partials = nullptr;  // [2*18][grid]
  double* res_out = nullptr;       // relative residual of the last sampled solve
  size_t ck_cap = 0, seg_cap = 0;
  // FP32 only: FP64 composition transport (remainder, rhs moment, iterates, diagonal)
  double *rC = nullptr, *fC = nullptr, *xCa = nullptr, *xCb = nullptr, *dlt = nullptr;
  double* partials = nullptr;
  DiagRecord* hist = nullptr;  // ring of per-step reductions
  DiagRecord* diag_now = nullptr;
  int32_t* first_bad = nullptr;
  int32_t* wet_flags = nullptr;  // [2] checks of felbm_set_wetting_device
  int64_t hist_cap = 16384;
  std::vector<double> host_omega;
  // internal orderings (see mesh_prep.hpp)
  std::vector<int32_t> node_perm, elem_perm;
  uint64_t perm_hash = 0;
  // timing
  bool timing = false;
  KStat kstat[K_COUNT];
  std::vector<PendingTiming> pending;
  std::vector<hipEvent_t> event_pool;
  std::vector<void*> allocations;
};

namespace {

thread_local std::string g_create_error;

int fail(felbm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_OK(c, call)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail((c), FELBM_EDEVICE, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
int dalloc(felbm_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return fail(c, FELBM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  c->allocations.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return FELBM_OK;
}

int dalloc_bytes(felbm_ctx* c, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 1));
  if (e != hipSuccess) return fail(c, FELBM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  c->allocations.push_back(*p);
  return FELBM_OK;
}

template <typename T>
int upload(felbm_ctx* c, T* dst, const std::vector<T>& src) {
  HIP_OK(c, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return FELBM_OK;
}

hipEvent_t take_event(felbm_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch a kernel on the context stream; with timing on, bracket it with
// events recorded by the command processor at kernel start and end.
template <typename F, typename... Args>
int launch_sm(felbm_ctx* c, int kid, F kernel, int grid, int block, uint32_t shmem, Args... args) {
  if (c->timing) {
    hipEvent_t s = take_event(c), t = take_event(c);
    if (!s || !t) return fail(c, FELBM_EDEVICE, "hipEventCreate failed");
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, c->stream, s, t, 0, args...);
    c->pending.push_back({kid, s, t});
  } else {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, c->stream, args...);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FELBM_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return FELBM_OK;
}

template <typename F, typename... Args>
int launch_bs(felbm_ctx* c, int kid, F kernel, int grid, int block, Args... args) {
  return launch_sm(c, kid, kernel, grid, block, 0u, args...);
}

template <typename F, typename... Args>
int launch(felbm_ctx* c, int kid, F kernel, int grid, Args... args) {
  return launch_sm(c, kid, kernel, grid, BLOCK, 0u, args...);
}

int harvest_timing(felbm_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    HIP_OK(c, hipEventSynchronize(p.stop));
    HIP_OK(c, hipEventElapsedTime(&ms, p.start, p.stop));
    c->kstat[p.kid].launches += 1;
    c->kstat[p.kid].total_ms += ms;
    c->event_pool.push_back(p.start);
    c->event_pool.push_back(p.stop);
  }
  c->pending.clear();
  return FELBM_OK;
}

// The checkpoints of a forward_ckpt run describe one trajectory; any call that
// changes the state or the wetting field discards them.
void invalidate_adjoint(felbm_ctx* c) {
  c->ck_steps = 0;
  c->ck_run = 0;
}

#define TRY(x)                   \
  do {                           \
    int r_ = (x);                \
    if (r_ != FELBM_OK) return r_; \
  } while (0)

// Algorithmic bytes per launch of each kernel (perfect reuse of gathered data)
void set_kernel_bytes(felbm_ctx* c) {
  const double N = (double)c->N, E = (double)c->E, s = (double)c->rs, nnz = (double)c->offdiag_nnz;
  const double pops = 18.0 * N * s;
  const double mat = nnz * (4.0 + s) + (double)(c->Np / 64 + 1) * 4.0;
  c->kstat[K_MOMENTS].bytes = 2 * pops + N * (8 + 3 * s) + N * 8 * 3;        // pop r/w, fields, mass + xy
  c->kstat[K_REDUCE].bytes = 0;
  c->kstat[K_GRAD].bytes = E * (12 + 56 + 16 + 2 * s) + N * (8 + s);
  c->kstat[K_EFLUX].bytes = E * (12 + 56 + 16 + 24);
  c->kstat[K_LAPC].bytes = N * (4 + 8 + 8 + 8 + 8 + 8 + 8 * 2 + 4 * 2) + 3 * E * (4 + 8);
  c->kstat[K_GRADMU].bytes = E * (12 + 48 + 16) + N * 8;
  c->kstat[K_LAPMU].bytes = E * (12 + 48 + 16 + 8);
  c->kstat[K_RHS].bytes = 2 * pops + N * (4 + 8 + 8 + 3 * s + 8) + 3 * E * 4 + E * (12 + 7 * s + 56 + 8);
  const double cons = c->prm.precision == FELBM_FP32 ? 8.0 * N : 0.0;  // one FP64 composition vector
  c->kstat[K_SWEEP_FIRST].bytes = 2 * pops + mat + 3 * cons;
  c->kstat[K_SWEEP_MID].bytes = 3 * pops + mat + 4 * cons;
  c->kstat[K_SWEEP_LAST].bytes = 4 * pops + mat + N + 5 * cons;
}

// How much of the field chain to compute: the time step's path (the
// precomputed operators: mu and lap mu only), the same with the nodal lap C
// kept for read-back, or the element-array chain (element gradients of C, p
// and mu, edge fluxes) that the adjoint and the nodal force scheme read.
enum FieldMode { FIELDS_STEP = 0, FIELDS_READ = 1, FIELDS_FULL = 2 };

FieldOps field_ops(felbm_ctx* c) {
  return FieldOps{c->lop_ptr, c->lop_col, c->lop_w, c->wptr, c->wab, c->wlen, c->eopp, c->ew};
}

template <typename real>
int enqueue_fields(felbm_ctx* c, bool collide, bool record, DiagRecord* rec_target, int mode) {
  const int gN = grid_for(c->N), gE = grid_for(c->E);
  const int N = (int)c->N, Np = (int)c->Np, E = (int)c->E;
  real* pop = (real*)c->pop;
  // the collision-step nodal scheme collides after its force fields (k_nc_collide)
  const bool nc = c->prm.force_scheme == FELBM_FORCES_NODAL_COLLIDE;
  if (collide && !nc)
    TRY(launch(c, K_MOMENTS, k_moments<real, true>, gN, pop, N, Np, c->sp, c->Cn, (real*)c->pn, (real*)c->uxn,
               (real*)c->uyn, (const double*)c->mass, (const double*)c->xy, c->band, (const double*)c->rC, c->partials));
  else
    TRY(launch(c, K_MOMENTS, k_moments<real, false>, gN, pop, N, Np, c->sp, c->Cn, (real*)c->pn, (real*)c->uxn,
               (real*)c->uyn, (const double*)c->mass, (const double*)c->xy, c->band, (const double*)c->rC, c->partials));
  if (record && !nc)
    TRY(launch_bs(c, K_REDUCE, k_reduce_final<>, 1, RBLOCK, (const double*)c->partials, gN, N, (int64_t)c->step, rec_target,
               c->first_bad));
  if (mode != FIELDS_FULL) {
    const FieldOps op = field_ops(c);
    if (mode == FIELDS_READ)
      TRY(launch(c, K_LAPC_OP, k_lapC_mu_op<real, true>, gN, N, op, (const double*)c->Cn, (const double*)c->bc, c->sp,
                 c->lapC, c->mu));
    else
      TRY(launch(c, K_LAPC_OP, k_lapC_mu_op<real, false>, gN, N, op, (const double*)c->Cn, (const double*)c->bc, c->sp,
                 c->lapC, c->mu));
    return launch(c, K_LAPMU_OP, k_lapmu_op, gE, E, (const int*)c->tri, op, (const double*)c->mu, c->lapmu);
  }
  TRY(launch(c, K_GRAD, k_elem_grad<real>, gE, E, (const int*)c->tri, (const double*)c->geo, (const double*)c->Cn,
             (const real*)c->pn, c->gC, (real*)c->gp));
  TRY(launch(c, K_EFLUX, k_edge_flux, gE, E, (const int*)c->tri, (const int*)c->enbr, (const double*)c->geo,
             (const double*)c->gC, (const double*)c->Cn, (const double*)c->bc, c->eflux));
  TRY(launch(c, K_LAPC, k_lapC_mu, gN, N, E, (const int*)c->n2e_ptr, (const int*)c->n2e, (const double*)c->eflux,
             (const double*)c->pvol, (const double*)c->Cn, (const double*)c->bc, (const int*)c->wall_nbr,
             (const double*)c->wall_len, c->sp, c->lapC, c->mu));
  TRY(launch(c, K_GRADMU, k_elem_gradmu, gE, E, (const int*)c->tri, (const double*)c->geo, (const double*)c->mu,
             c->gmu));
  if (c->prm.force_scheme == FELBM_FORCES_NODAL)
    return launch(c, K_NODEF, k_node_forces<real>, gN, N, Np, E, (const int*)c->n2e_ptr, (const int*)c->n2e,
                  (const int*)c->enbr, (const double*)c->geo, (const double*)c->pvol, (const double*)c->gC,
                  (const real*)c->gp, (const double*)c->gmu, (const double*)c->Cn, (const real*)c->uxn,
                  (const real*)c->uyn, (const double*)c->mu, c->sp, (real*)c->Fn);
  if (nc) {
    // half-force moments of psi_bar (velocity and pressure), nodal lap mu, the
    // reductions of the corrected fields; then grad p of the corrected pressure
    TRY(launch(c, K_NODEF, k_nc_fields<real, true>, gN, N, E, (const int*)c->n2e_ptr, (const int*)c->n2e,
               (const int*)c->enbr, (const double*)c->geo, (const double*)c->pvol, (const double*)c->gC,
               (const double*)c->gmu, (const double*)c->Cn, (const double*)c->mu, (const uint8_t*)c->is_wall, c->sp,
               (real*)c->pn, (real*)c->uxn, (real*)c->uyn, c->lapmu_n, (const double*)c->mass, (const double*)c->xy,
               c->band, c->partials));
    if (record)
      TRY(launch_bs(c, K_REDUCE, k_reduce_final<>, 1, RBLOCK, (const double*)c->partials, gN, N, (int64_t)c->step,
                    rec_target, c->first_bad));
    TRY(launch(c, K_GRAD, k_elem_grad<real>, gE, E, (const int*)c->tri, (const double*)c->geo, (const double*)c->Cn,
               (const real*)c->pn, c->gC, (real*)c->gp));
    if (collide)
      TRY(launch(c, K_NODEF, k_nc_collide<real, false>, gN, N, Np, E, (const int*)c->n2e_ptr, (const int*)c->n2e,
                 (const double*)c->geo, (const double*)c->pvol, (const double*)c->gC, (const real*)c->gp,
                 (const double*)c->Cn, (const real*)c->pn, (const real*)c->uxn, (const real*)c->uyn,
                 (const double*)c->mu, (const double*)c->lapmu_n, (const uint8_t*)c->is_wall, c->sp, pop));
    return FELBM_OK;
  }
  TRY(launch(c, K_LAPMU, k_elem_lapmu, gE, E, (const int*)c->enbr, (const double*)c->geo, (const double*)c->gmu,
             c->lapmu));
  return FELBM_OK;
}

template <typename real>
int enqueue_rhs(felbm_ctx* c) {
  const int gN = grid_for(c->N);
  const int N = (int)c->N, Np = (int)c->Np, E = (int)c->E;
  if (c->prm.force_scheme == FELBM_FORCES_NODAL)
    return launch(c, K_RHS, k_rhs_nodal<real, true>, gN, N, Np, E, (const int*)c->n2e_ptr, (const int*)c->n2e,
                  (const int*)c->tri, (const double*)c->geo, (const real*)c->Fn, (const real*)c->pop,
                  (const double*)c->mass, c->sp, (real*)c->f);
  if (c->prm.force_scheme == FELBM_FORCES_NODAL_COLLIDE)  // the force acted in the collision
    return launch(c, K_RHS, k_rhs_nodal<real, false>, gN, N, Np, E, (const int*)c->n2e_ptr, (const int*)c->n2e,
                  (const int*)c->tri, (const double*)c->geo, (const real*)nullptr, (const real*)c->pop,
                  (const double*)c->mass, c->sp, (real*)c->f);
  if (c->use_rhs_lds) {
    TileArgs ta{c->tile_off, c->tslot, c->halo_off, c->halo, c->ntiles, c->tile_slots};
    const int grid = (c->ntiles + 7) / 8 * 8;
    return launch_sm(c, K_RHS, k_rhs_lds<real>, grid, BLOCK, rhs_lds_bytes<real>(), N, Np, E, ta,
                     RhsTile{c->rhs_off, c->rhs_ent, c->gaos, c->lapmu}, (const double*)c->Cn, (const real*)c->pn,
                     (const real*)c->uxn, (const real*)c->uyn, (const double*)c->mu, (const real*)c->pop,
                     (const double*)c->mass, c->sp, (real*)c->f, c->fC);
  }
  return launch(c, K_RHS, k_rhs<real>, gN, N, Np, E, (const int*)c->n2e_ptr, (const int*)c->n2e, (const int*)c->tri,
                (const real*)c->geor, (const double*)c->geo, (const real*)c->pn,
                (const double*)c->lapmu, (const double*)c->Cn, (const real*)c->uxn, (const real*)c->uyn,
                (const double*)c->mu, (const real*)c->pop, (const double*)c->mass, c->sp, (real*)c->f, c->fC);
}

template <typename real, int MODE>
int sweep(felbm_ctx* c, int kid, const real* xin, real* xout, real w, const ConsArgs& cs,
          const real* fsrc = nullptr) {
  const int N = (int)c->N, Np = (int)c->Np;
  real* pop = (real*)c->pop;
  const real* f = fsrc ? fsrc : (const real*)c->f;
  if (c->use_lds) {
    TileArgs ta{c->tile_off, c->tslot, c->halo_off, c->halo, c->ntiles, c->tile_slots};
    return launch_sm(c, kid, k_sweep_dma<real, MODE>, (2 * c->ntiles + 7) / 8 * 8, BLOCK, sweep_dma_lds_bytes<real>(),
                     N, Np, ta, (const real*)c->tval, f, xin, xout, pop, (const uint8_t*)c->is_wall, w, cs);
  }
  return launch(c, kid, k_sweep<real, MODE>, grid_for(c->N), N, Np, (const int*)c->sell_ptr, (const int*)c->sell_col,
                (const real*)c->sell_val, f, xin, xout, pop, (const uint8_t*)c->is_wall, w, cs);
}

// Residual of the solve: M-weighted norms of (A x - f) and f per population,
// reduced in FP64 into c->res_out.
template <typename real>
int enqueue_residual(felbm_ctx* c, const real* x) {
  const int gN = grid_for(c->N);
  TRY(launch(c, K_RESID, k_residual<real>, gN, (int)c->N, (int)c->Np, (const int*)c->sell_ptr, (const int*)c->sell_col,
             (const real*)c->sell_val, (const real*)c->f, x, (const double*)c->mass, c->res_partials));
  return launch_bs(c, K_RESID, k_residual_final, 1, RBLOCK_RES, (const double*)c->res_partials, gN, c->res_out);
}

// The solve of a step whose residual is sampled: all K sweeps write their
// iterate, the residual of x_K is reduced, then the update psi_hat + x_K and
// the wall operator run as the no-sweep form with x_K (and its FP64
// composition part) in place of f.  Bitwise the same update as the fused
// last sweep.
template <typename real>
int enqueue_solve_sampled(felbm_ctx* c) {
  const int K = c->prm.solver_sweeps;
  real *xin = (real*)c->f, *xout = (real*)c->xa, *spare = (real*)c->xb;
  double *cin = c->fC, *cout = c->xCa, *cspare = c->xCb;
  ConsArgs cs{c->fC, nullptr, nullptr, c->dlt, c->Cn, c->rC, 0.0};
  for (int j = 0; j < K; ++j) {
    cs.w = c->cheb_w[j];
    cs.xCin = cin;
    cs.xCout = cout;
    if (j == 0)
      TRY((sweep<real, 0>(c, K_SWEEP_FIRST, nullptr, xout, (real)c->cheb_w[0], cs)));
    else
      TRY((sweep<real, 1>(c, K_SWEEP_MID, xin, xout, (real)c->cheb_w[j], cs)));
    // the next sweep reads this iterate; the other buffer receives the next one
    real* nx = j == 0 ? spare : xin;
    double* ncx = j == 0 ? cspare : cin;
    xin = xout;
    cin = cout;
    xout = nx;
    cout = ncx;
  }
  TRY(enqueue_residual<real>(c, xin));
  ConsArgs fin{cin, nullptr, nullptr, c->dlt, c->Cn, c->rC, 0.0};
  return sweep<real, 4>(c, K_SWEEP_LAST, nullptr, nullptr, (real)0, fin, xin);
}

// K Chebyshev-step Richardson sweeps on f, then psi_bar^{n+1} = psi_hat + x_K
// and the wall operator (fused into the last sweep)
template <typename real>
int enqueue_solve(felbm_ctx* c) {
  const int K = c->prm.solver_sweeps;
  if (c->residual_every > 0 && c->step % c->residual_every == 0) {
    c->residual_step = c->step;
    return enqueue_solve_sampled<real>(c);
  }
  real *xa = (real*)c->xa, *xb = (real*)c->xb;
  ConsArgs cs{c->fC, nullptr, nullptr, c->dlt, c->Cn, c->rC, 0.0};
  if (K == 0) return sweep<real, 4>(c, K_SWEEP_LAST, nullptr, nullptr, (real)0, cs);
  cs.w = c->cheb_w[0];
  if (K == 1) return sweep<real, 3>(c, K_SWEEP_LAST, nullptr, nullptr, (real)c->cheb_w[0], cs);
  cs.xCout = c->xCa;
  TRY((sweep<real, 0>(c, K_SWEEP_FIRST, nullptr, xa, (real)c->cheb_w[0], cs)));
  real *xin = xa, *xout = xb;
  double *cin = c->xCa, *cout = c->xCb;
  for (int j = 1; j < K - 1; ++j) {
    cs.w = c->cheb_w[j];
    cs.xCin = cin;
    cs.xCout = cout;
    TRY((sweep<real, 1>(c, K_SWEEP_MID, xin, xout, (real)c->cheb_w[j], cs)));
    std::swap(xin, xout);
    std::swap(cin, cout);
  }
  cs.w = c->cheb_w[K - 1];
  cs.xCin = cin;
  cs.xCout = nullptr;
  return sweep<real, 2>(c, K_SWEEP_LAST, xin, nullptr, (real)c->cheb_w[K - 1], cs);
}

int step_field_mode(const felbm_ctx* c) {
  return c->prm.force_scheme == FELBM_FORCES_MIXED ? FIELDS_STEP : FIELDS_FULL;
}

int read_field_mode(const felbm_ctx* c) {
  return c->prm.force_scheme == FELBM_FORCES_MIXED ? FIELDS_READ : FIELDS_FULL;
}

// Initial state of the collision-step nodal scheme: psi_bar^0 = psi_eq - dt/2 F
// with F from the initial fields (the populations hold psi_eq on entry).
template <typename real>
int enqueue_nc_init(felbm_ctx* c) {
  const int gN = grid_for(c->N), gE = grid_for(c->E);
  const int N = (int)c->N, Np = (int)c->Np, E = (int)c->E;
  real* pop = (real*)c->pop;
  TRY(launch(c, K_MOMENTS, k_moments<real, false>, gN, pop, N, Np, c->sp, c->Cn, (real*)c->pn, (real*)c->uxn,
             (real*)c->uyn, (const double*)c->mass, (const double*)c->xy, c->band, (const double*)c->rC, c->partials));
  TRY(launch(c, K_GRAD, k_elem_grad<real>, gE, E, (const int*)c->tri, (const double*)c->geo, (const double*)c->Cn,
             (const real*)c->pn, c->gC, (real*)c->gp));
  TRY(launch(c, K_EFLUX, k_edge_flux, gE, E, (const int*)c->tri, (const int*)c->enbr, (const double*)c->geo,
             (const double*)c->gC, (const double*)c->Cn, (const double*)c->bc, c->eflux));
  TRY(launch(c, K_LAPC, k_lapC_mu, gN, N, E, (const int*)c->n2e_ptr, (const int*)c->n2e, (const double*)c->eflux,
             (const double*)c->pvol, (const double*)c->Cn, (const double*)c->bc, (const int*)c->wall_nbr,
             (const double*)c->wall_len, c->sp, c->lapC, c->mu));
  TRY(launch(c, K_GRADMU, k_elem_gradmu, gE, E, (const int*)c->tri, (const double*)c->geo, (const double*)c->mu,
             c->gmu));
  TRY(launch(c, K_NODEF, k_nc_fields<real, false>, gN, N, E, (const int*)c->n2e_ptr, (const int*)c->n2e,
             (const int*)c->enbr, (const double*)c->geo, (const double*)c->pvol, (const double*)c->gC,
             (const double*)c->gmu, (const double*)c->Cn, (const double*)c->mu, (const uint8_t*)c->is_wall, c->sp,
             (real*)c->pn, (real*)c->uxn, (real*)c->uyn, c->lapmu_n, (const double*)c->mass, (const double*)c->xy,
             c->band, c->partials));
  return launch(c, K_NODEF, k_nc_collide<real, true>, gN, N, Np, E, (const int*)c->n2e_ptr, (const int*)c->n2e,
                (const double*)c->geo, (const double*)c->pvol, (const double*)c->gC, (const real*)c->gp,
                (const double*)c->Cn, (const real*)c->pn, (const real*)c->uxn, (const real*)c->uyn,
                (const double*)c->mu, (const double*)c->lapmu_n, (const uint8_t*)c->is_wall, c->sp, pop);
}

template <typename real>
int enqueue_step(felbm_ctx* c) {
  TRY(enqueue_fields<real>(c, true, true, c->hist + (c->step % c->hist_cap), step_field_mode(c)));
  TRY(enqueue_rhs<real>(c));
  TRY(enqueue_solve<real>(c));
  c->step += 1;
  return FELBM_OK;
}

int enqueue_steps(felbm_ctx* c, int64_t n) {
  for (int64_t s = 0; s < n; ++s) {
    if (c->prm.precision == FELBM_FP64)
      TRY(enqueue_step<double>(c));
    else
      TRY(enqueue_step<float>(c));
  }
  return FELBM_OK;
}

int enqueue_fields_any(felbm_ctx* c, bool collide, bool record, DiagRecord* target, int mode) {
  return c->prm.precision == FELBM_FP64 ? enqueue_fields<double>(c, collide, record, target, mode)
                                        : enqueue_fields<float>(c, collide, record, target, mode);
}

int to_double(felbm_ctx* c, const void* src, double* dst_dev, int64_t n) {
  const int g = (int)((n + BLOCK - 1) / BLOCK);
  if (c->prm.precision == FELBM_FP64)
    HIP_OK(c, hipMemcpyAsync(dst_dev, src, n * 8, hipMemcpyDeviceToDevice, c->stream));
  else
    hipLaunchKernelGGL(k_to_double<float>, dim3(g), dim3(BLOCK), 0, c->stream, (int)n, (const float*)src, dst_dev);
  HIP_OK(c, hipGetLastError());
  return FELBM_OK;
}

// Copy a [18][Np] device population array to a host [18][N] double array.
int copy_pops_out(felbm_ctx* c, const void* dev, double* out) {
  double* tmp = nullptr;
  HIP_OK(c, hipMallocAsync((void**)&tmp, 18 * c->Np * sizeof(double), c->stream));
  int r = to_double(c, dev, tmp, 18 * c->Np);
  std::vector<double> host(18 * c->Np);
  if (r == FELBM_OK) {
    hipError_t e = hipMemcpyAsync(host.data(), tmp, host.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) r = fail(c, FELBM_EDEVICE, std::string("population copy failed: ") + hipGetErrorString(e));
  }
  if (r == FELBM_OK)
    for (int64_t a = 0; a < 18; ++a)
      for (int64_t k = 0; k < c->N; ++k) out[a * c->N + c->node_perm[k]] = host[a * c->Np + k];
  (void)hipFreeAsync(tmp, c->stream);
  (void)hipStreamSynchronize(c->stream);
  return r;
}

std::vector<double> chebyshev_steps(int K, double lo, double hi) {
  // roots of T_K mapped to [lo, hi], taken alternately from the top and the
  // bottom of the spectrum so that partial products stay bounded
  std::vector<double> lam(K), out;
  for (int i = 0; i < K; ++i) lam[i] = 0.5 * (hi + lo) + 0.5 * (hi - lo) * std::cos((2.0 * i + 1.0) * M_PI / (2.0 * K));
  int i = 0, j = K - 1;
  while (i <= j) {
    out.push_back(1.0 / lam[i]);
    if (i != j) out.push_back(1.0 / lam[j]);
    ++i;
    --j;
  }
  return out;
}

// ---------------------------------------------------------------------------
// adjoint (reverse pass) of the step, with checkpoints
// ---------------------------------------------------------------------------
size_t dev_state_bytes(const felbm_ctx* c) {
  return (size_t)18 * c->Np * c->rs + (c->prm.precision == FELBM_FP32 ? (size_t)c->Np * 8 : 0);
}

int state_to(felbm_ctx* c, void* dst) {
  const size_t pb = (size_t)18 * c->Np * c->rs;
  HIP_OK(c, hipMemcpyAsync(dst, c->pop, pb, hipMemcpyDeviceToDevice, c->stream));
  if (c->rC) HIP_OK(c, hipMemcpyAsync((char*)dst + pb, c->rC, c->Np * 8, hipMemcpyDeviceToDevice, c->stream));
  return FELBM_OK;
}

int state_from(felbm_ctx* c, const void* src) {
  const size_t pb = (size_t)18 * c->Np * c->rs;
  HIP_OK(c, hipMemcpyAsync(c->pop, src, pb, hipMemcpyDeviceToDevice, c->stream));
  if (c->rC) HIP_OK(c, hipMemcpyAsync(c->rC, (const char*)src + pb, c->Np * 8, hipMemcpyDeviceToDevice, c->stream));
  return FELBM_OK;
}

int ensure_adjoint_buffers(felbm_ctx* c) {
  if (c->lam) return FELBM_OK;
  const size_t pb = (size_t)18 * c->Np * c->rs;
  TRY(dalloc_bytes(c, &c->lam, pb));
  TRY(dalloc_bytes(c, &c->lhat, pb));
  TRY(dalloc(c, &c->ea, (size_t)EA_N * c->E));
  TRY(dalloc_bytes(c, &c->lqe, (size_t)18 * c->E * c->rs));
  TRY(dalloc(c, &c->lgmu, 2 * c->E));
  TRY(dalloc(c, &c->lgC, 2 * c->E));
  TRY(dalloc(c, &c->lmu, c->Np));
  TRY(dalloc(c, &c->gomega, c->Np));
  return FELBM_OK;
}

AdjGeom adj_geom(felbm_ctx* c) {
  return AdjGeom{c->tri,  c->enbr,     c->erev, c->geo, c->n2e_ptr, c->n2e,     c->mass,
                 c->wall_nbr, c->wall_len, c->bc, c->is_wall, (int)c->N, (int)c->Np, (int)c->E};
}

// transpose of the solve: the same K sweeps applied to f = (W lam)/m, result returned
template <typename real>
int enqueue_adjoint_solve(felbm_ctx* c, real** result) {
  const int K = c->prm.solver_sweeps;
  real *xa = (real*)c->xa, *xb = (real*)c->xb;
  if (K == 0) {
    HIP_OK(c, hipMemcpyAsync(xa, c->f, (size_t)18 * c->Np * c->rs, hipMemcpyDeviceToDevice, c->stream));
    *result = xa;
    return FELBM_OK;
  }
  // the FP32 sweeps also carry the FP64 composition scalar: run it on zeros
  if (c->fC) HIP_OK(c, hipMemsetAsync(c->fC, 0, c->Np * 8, c->stream));
  ConsArgs cs{c->fC, nullptr, c->xCa, c->dlt, c->Cn, nullptr, c->cheb_w[0]};
  const std::vector<double>& w = c->cheb_w;
  real *cur = xa, *nxt = xb;
  double *ccur = c->xCa, *cnxt = c->xCb;
  TRY((sweep<real, 0>(c, K_SWEEP_FIRST, nullptr, cur, (real)w[0], cs)));
  for (int j = 1; j < K; ++j) {
    cs.w = w[j];
    cs.xCin = ccur;
    cs.xCout = cnxt;
    TRY((sweep<real, 1>(c, K_SWEEP_MID, cur, nxt, (real)w[j], cs)));
    std::swap(cur, nxt);
    std::swap(ccur, cnxt);
  }
  *result = cur;
  return FELBM_OK;
}

// one reverse step: lam (= dL/dpsi_bar^{n+1}) -> dL/dpsi_bar^n, gomega += dL/dOmega_c.
// Requires psi_bar^n in pop and its forward fields recomputed.
template <typename real>
int enqueue_adjoint_step(felbm_ctx* c) {
  const int gN = grid_for(c->N), gE = grid_for(c->E);
  AdjGeom g = adj_geom(c);
  real* lam = (real*)c->lam;
  TRY(launch(c, K_ADJ_PREP, k_adj_prep<real>, gN, g, (const real*)lam, (real*)c->f));
  real* lb = nullptr;
  TRY(enqueue_adjoint_solve<real>(c, &lb));
  TRY(launch(c, K_ADJ_FORCE, k_adj_force<real>, gE, g, c->sp, (const real*)lb, (const double*)c->Cn,
             (const real*)c->uxn, (const real*)c->uyn, (const double*)c->mu, (const double*)c->gC, (const real*)c->gp,
             (const double*)c->lapmu, c->ea, (real*)c->lqe));
  TRY(launch(c, K_ADJ_STREAM, k_adj_stream<real>, gN, g, (const real*)lam, (const real*)c->lqe, (real*)c->lhat));
  TRY(launch(c, K_ADJ_GMU, k_adj_gmu, gE, g, (const double*)c->ea, c->lgmu));
  TRY(launch(c, K_ADJ_MU, k_adj_mu, gN, g, (const double*)c->ea, (const double*)c->lgmu, c->lmu));
  TRY(launch(c, K_ADJ_GC, k_adj_gC, gE, g, c->sp, (const double*)c->ea, (const double*)c->lmu, c->lgC));
  const double bc_scale = c->sp.kappa > 0 ? std::sqrt(2.0 * c->sp.kappa * c->sp.beta) / c->sp.kappa : 0.0;
  TRY(launch(c, K_ADJ_NODE, k_adj_node<real>, gN, g, c->sp, bc_scale, (const real*)c->pop, (const double*)c->Cn,
             (const real*)c->pn, (const real*)c->uxn, (const real*)c->uyn, (const double*)c->ea,
             (const double*)c->lgC, (const double*)c->lmu, (const real*)c->lhat, lam, c->gomega));
  return FELBM_OK;
}

int enqueue_adjoint_step_any(felbm_ctx* c) {
  return c->prm.precision == FELBM_FP64 ? enqueue_adjoint_step<double>(c) : enqueue_adjoint_step<float>(c);
}

// The precomputed operators of the chemical-potential chain, assembled in FP64
// from the element geometry: the node rows of the patch Laplacian of C with
// averaged outer-edge gradients (eqn:lapl_int_mp) divided by the patch
// volume, the wall edges of each patch (eq. bc2 flux), and the six weights of
// the element Laplacian of mu (Sec. II.D).  Stored in the working precision.
template <typename wreal>
int build_field_operators(felbm_ctx* c, const MeshPrep& m, const std::vector<double>& pvol) {
  const int64_t N = m.N, Np = m.Np, E = m.E;
  auto A = [&](int64_t e) { return m.geo[e]; };
  auto gx = [&](int64_t e, int v) { return m.geo[(1 + 2 * v) * E + e]; };
  auto gy = [&](int64_t e, int v) { return m.geo[(2 + 2 * v) * E + e]; };
  // node rows: (column, weight) in first-appearance order, own node dropped
  std::vector<int32_t> rptr(N + 1, 0), rcol;
  std::vector<double> rval;
  std::vector<int32_t> wptr(N + 1, 0);
  std::vector<int2> wab;
  std::vector<double> wlen;
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t k = 0; k < N; ++k) {
    row.clear();
    auto add = [&](int32_t node, double w) {
      for (auto& pr : row)
        if (pr.first == node) {
          pr.second += w;
          return;
        }
      row.push_back({node, w});
    };
    const double iv = 1.0 / pvol[k];
    for (int32_t q = m.n2e_ptr[k]; q < m.n2e_ptr[k + 1]; ++q) {
      const int64_t e = m.n2e[q] >> 2;
      const int l = m.n2e[q] & 3;
      const int64_t nb = m.enbr[l * E + e];
      if (nb >= 0) {
        // -2 A_e grad N_l . (grad C_e + grad C_nb) / 2
        for (int v = 0; v < 3; ++v)
          add(m.tri[v * E + e], -A(e) * (gx(e, l) * gx(e, v) + gy(e, l) * gy(e, v)) * iv);
        for (int v = 0; v < 3; ++v)
          add(m.tri[v * E + nb], -A(e) * (gx(e, l) * gx(nb, v) + gy(e, l) * gy(nb, v)) * iv);
      } else {
        const int32_t a = m.tri[((l + 1) % 3) * E + e], b = m.tri[((l + 2) % 3) * E + e];
        wab.push_back(int2{a, b});
        wlen.push_back(2.0 * A(e) * std::sqrt(gx(e, l) * gx(e, l) + gy(e, l) * gy(e, l)) * iv);
      }
    }
    for (int w = 0; w < 2; ++w) {
      const int32_t j = m.wall_nbr[w * N + k];
      if (j >= 0) {
        wab.push_back(int2{(int32_t)k, j});
        wlen.push_back(m.wall_len[w * N + k] * iv);
      }
    }
    wptr[k + 1] = (int32_t)wab.size();
    for (auto& pr : row)
      if (pr.first != (int32_t)k) {
        rcol.push_back(pr.first);
        rval.push_back(pr.second);
      }
    rptr[k + 1] = (int32_t)rcol.size();
  }
  // sliced ELL, slice height 64, padded with the node itself and weight 0
  const int64_t nslices = Np / 64;
  std::vector<int32_t> sptr(nslices + 1, 0), scol;
  std::vector<wreal> sval;
  int64_t true_nnz = 0;
  for (int64_t sl = 0; sl < nslices; ++sl) {
    int64_t width = 0;
    for (int64_t i = sl * 64; i < std::min<int64_t>(N, (sl + 1) * 64); ++i) width = std::max<int64_t>(width, rptr[i + 1] - rptr[i]);
    const size_t base = scol.size();
    scol.resize(base + width * 64);
    sval.resize(base + width * 64);
    for (int64_t q = 0; q < width; ++q)
      for (int lane = 0; lane < 64; ++lane) {
        const int64_t i = sl * 64 + lane, idx = base + q * 64 + lane;
        const bool real_entry = i < N && q < rptr[i + 1] - rptr[i];
        scol[idx] = real_entry ? rcol[rptr[i] + q] : (int32_t)std::min<int64_t>(i, N - 1);
        sval[idx] = real_entry ? (wreal)rval[rptr[i] + q] : (wreal)0;
        true_nnz += real_entry;
      }
    sptr[sl + 1] = (int32_t)scol.size();
  }
  // element rows: weights of mu_1 - mu_0, mu_2 - mu_0 and of the three vertices across the edges
  std::vector<int32_t> eopp(3 * E);
  std::vector<double> ew(5 * E);
  for (int64_t e = 0; e < E; ++e) {
    double wv[3] = {0, 0, 0}, wo[3] = {0, 0, 0};
    int32_t opp[3] = {m.tri[e], m.tri[e], m.tri[e]};
    for (int l = 0; l < 3; ++l) {
      const int64_t nb = m.enbr[l * E + e];
      if (nb < 0) continue;  // zero normal flux of grad mu through a wall (eqn:bc1)
      for (int v = 0; v < 3; ++v) wv[v] -= gx(e, l) * gx(e, v) + gy(e, l) * gy(e, v);
      for (int w = 0; w < 3; ++w) {
        const int32_t node = m.tri[w * E + nb];
        const double wt = -(gx(e, l) * gx(nb, w) + gy(e, l) * gy(nb, w));
        int v = 0;
        while (v < 3 && m.tri[v * E + e] != node) ++v;
        if (v < 3) {
          wv[v] += wt;
        } else {
          opp[l] = node;
          wo[l] += wt;
        }
      }
    }
    ew[e] = wv[1];
    ew[E + e] = wv[2];
    for (int l = 0; l < 3; ++l) {
      eopp[l * E + e] = opp[l];
      ew[(2 + l) * E + e] = wo[l];
    }
  }
  TRY(dalloc(c, &c->lop_ptr, sptr.size()));
  TRY(dalloc(c, &c->lop_col, scol.size()));
  TRY(dalloc_bytes(c, &c->lop_w, sval.size() * sizeof(wreal)));
  TRY(dalloc(c, &c->wptr, wptr.size()));
  TRY(dalloc(c, &c->wab, std::max<size_t>(wab.size(), 1)));
  TRY(dalloc(c, &c->wlen, std::max<size_t>(wlen.size(), 1)));
  TRY(dalloc(c, &c->eopp, eopp.size()));
  TRY(dalloc_bytes(c, &c->ew, ew.size() * sizeof(double)));
  TRY(upload(c, c->lop_ptr, sptr));
  TRY(upload(c, c->lop_col, scol));
  HIP_OK(c, hipMemcpyAsync(c->lop_w, sval.data(), sval.size() * sizeof(wreal), hipMemcpyHostToDevice, c->stream));
  TRY(upload(c, c->wptr, wptr));
  if (!wab.empty()) {
    TRY(upload(c, c->wab, wab));
    TRY(upload(c, c->wlen, wlen));
  }
  TRY(upload(c, c->eopp, eopp));
  HIP_OK(c, hipMemcpyAsync(c->ew, ew.data(), ew.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));  // host vectors are about to go out of scope
  // algorithmic bytes: true entries (column + weight), C_k, the wall pointer, mu written;
  // per element three vertex ids, three opposite ids, five weights, lap mu written
  const double ws = (double)sizeof(wreal);
  c->kstat[K_LAPC_OP].bytes = (double)true_nnz * (4 + ws) + (double)N * (8 + 4 + 8) + (double)wab.size() * (8 + 8);
  c->kstat[K_LAPMU_OP].bytes = (double)E * (12 + 12 + 5 * 8 + 8) + (double)N * 8;
  return FELBM_OK;
}

// Per-tile incident-element entries of the LDS-staged right-hand side:
// for node lane of tile t, entry k = (element * 4 + local vertex, LDS slots of
// the element's three vertices), column-major per tile, padded with -1.  Every
// vertex of an element incident to a tile node is a tile node or in the tile's
// halo (the halo lists every node coupled by the mass matrix).
int build_rhs_tiles(felbm_ctx* c, const MeshPrep& m, const std::vector<int32_t>& halo_off,
                    const std::vector<int32_t>& halo) {
  const int64_t N = m.N, E = m.E, nt = (N + TILE - 1) / TILE;
  std::vector<int32_t> off(nt + 1, 0);
  std::vector<int2> ent;
  int64_t true_entries = 0;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t lo = t * TILE, hi = std::min<int64_t>(N, lo + TILE);
    const int32_t* hb = halo.data() + halo_off[t];
    const int32_t* he = halo.data() + halo_off[t + 1];
    int64_t width = 0;
    for (int64_t i = lo; i < hi; ++i) width = std::max<int64_t>(width, m.n2e_ptr[i + 1] - m.n2e_ptr[i]);
    const size_t base = ent.size();
    ent.resize(base + width * TILE, int2{-1, 0});
    for (int64_t i = lo; i < hi; ++i) {
      const int64_t lane = i - lo;
      for (int32_t q = m.n2e_ptr[i], k = 0; q < m.n2e_ptr[i + 1]; ++q, ++k) {
        const int32_t packed = m.n2e[q], e = packed >> 2;
        int32_t slots = 0;
        for (int v = 0; v < 3; ++v) {
          const int32_t node = m.tri[v * E + e];
          int32_t sl;
          if (node >= lo && node < hi) {
            sl = (int32_t)(node - lo);
          } else {
            const int32_t* p = std::lower_bound(hb, he, node);
            if (p == he || *p != node) return FELBM_OK;  // keep the global-gather kernel
            sl = (int32_t)(TILE + (p - hb));
          }
          slots |= sl << (9 * v);
        }
        ent[base + k * TILE + lane] = int2{packed, slots};
        ++true_entries;
      }
    }
    off[t + 1] = (int32_t)ent.size();
  }
  // element record {dN1/dx, dN1/dy, dN2/dx, dN2/dy}: grad N0 = -(grad N1 + grad N2)
  // and A = 1 / (2 det[grad N1; grad N2]) follow in the kernel
  std::vector<double> gaos(4 * (size_t)E, 0.0);
  for (int64_t e = 0; e < E; ++e)
    for (int q = 0; q < 4; ++q) gaos[4 * e + q] = m.geo[(3 + q) * E + e];
  TRY(dalloc(c, &c->rhs_off, off.size()));
  TRY(dalloc(c, &c->rhs_ent, ent.size()));
  TRY(dalloc(c, &c->gaos, gaos.size()));
  TRY(upload(c, c->rhs_off, off));
  TRY(upload(c, c->rhs_ent, ent));
  TRY(upload(c, c->gaos, gaos));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->use_rhs_lds = true;
  // algorithmic bytes: populations and nodal fields once per node (C, mu, u, p, mass),
  // f (and, FP32, fC) written, the true entries, element data (FP64 geometry, lap mu)
  const double Nd = (double)N, Ed = (double)E;
  const double s = (double)c->rs, cons = c->prm.precision == FELBM_FP32 ? 8.0 : 0.0;
  c->kstat[K_RHS].bytes = 2 * 18 * Nd * s + Nd * (8 + 8 + 3 * s + 8 + cons) + (double)true_entries * 8 +
                          Ed * (32 + 8) + (double)halo.size() * 4;
  return FELBM_OK;
}

// Per-tile halo lists and local-slot matrix rows for the LDS-staged sweep.
// Falls back to the global sliced-ELL sweep when a tile row is wider than
// MAXW or a tile's halo has more than HALO_MAX nodes.
int build_tiles(felbm_ctx* c, const MeshPrep& m) {
  const int64_t N = m.N, nt = (N + TILE - 1) / TILE;
  std::vector<int32_t> tile_off(nt + 1, 0), halo_off(nt + 1, 0), halo;
  std::vector<uint16_t> slot;
  std::vector<double> val;
  int64_t maxh = 0;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t lo = t * TILE, hi = std::min<int64_t>(N, lo + TILE);
    std::vector<int32_t> hl;
    int64_t width = 0;
    for (int64_t i = lo; i < hi; ++i) {
      width = std::max<int64_t>(width, m.csr_ptr[i + 1] - m.csr_ptr[i]);
      for (int32_t q = m.csr_ptr[i]; q < m.csr_ptr[i + 1]; ++q)
        if (m.csr_col[q] < lo || m.csr_col[q] >= hi) hl.push_back(m.csr_col[q]);
    }
    std::sort(hl.begin(), hl.end());
    hl.erase(std::unique(hl.begin(), hl.end()), hl.end());
    if (width > MAXW) return FELBM_OK;  // keep the sliced-ELL sweep
    maxh = std::max<int64_t>(maxh, (int64_t)hl.size());
    const size_t base = slot.size();
    slot.resize(base + width * TILE);
    val.resize(base + width * TILE);
    for (int64_t k = 0; k < width; ++k)
      for (int lane = 0; lane < TILE; ++lane) {
        const int64_t i = lo + lane, idx = base + k * TILE + lane;
        slot[idx] = (uint16_t)lane;
        val[idx] = 0.0;
        if (i < hi && k < m.csr_ptr[i + 1] - m.csr_ptr[i]) {
          const int32_t j = m.csr_col[m.csr_ptr[i] + k];
          const int64_t s = (j >= lo && j < hi) ? j - lo
                                                  : TILE + (std::lower_bound(hl.begin(), hl.end(), j) - hl.begin());
          slot[idx] = (uint16_t)s;
          val[idx] = m.csr_val[m.csr_ptr[i] + k];
        }
      }
    tile_off[t + 1] = (int32_t)slot.size();
    halo.insert(halo.end(), hl.begin(), hl.end());
    halo_off[t + 1] = (int32_t)halo.size();
  }
  if (maxh > HALO_MAX) return FELBM_OK;  // keep the sliced-ELL sweep
  const int64_t slots = TILE + maxh;
  TRY(dalloc(c, &c->tile_off, tile_off.size()));
  TRY(dalloc(c, &c->halo_off, halo_off.size()));
  TRY(dalloc(c, &c->halo, halo.size()));
  TRY(dalloc(c, &c->tslot, slot.size()));
  TRY(dalloc_bytes(c, &c->tval, val.size() * c->rs));
  TRY(upload(c, c->tile_off, tile_off));
  TRY(upload(c, c->halo_off, halo_off));
  TRY(upload(c, c->halo, halo));
  TRY(upload(c, c->tslot, slot));
  if (c->prm.precision == FELBM_FP64) {
    TRY(upload(c, (double*)c->tval, val));
  } else {
    std::vector<float> v32(val.begin(), val.end());
    TRY(upload(c, (float*)c->tval, v32));
    HIP_OK(c, hipStreamSynchronize(c->stream));
  }
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->ntiles = (int)nt;
  c->tile_slots = (int)slots;
  c->use_lds = true;
  // algorithmic bytes: true nonzeros only (padding entries are not counted)
  const double s = (double)c->rs, Nd = (double)N;
  const double tmat = (double)m.offdiag_nnz * (2.0 + s) + (double)halo.size() * 4.0;
  const double cons = c->prm.precision == FELBM_FP32 ? 8.0 * Nd : 0.0;
  c->kstat[K_SWEEP_FIRST].bytes = 2 * 18 * Nd * s + tmat + 3 * cons;
  c->kstat[K_SWEEP_MID].bytes = 3 * 18 * Nd * s + tmat + 4 * cons;
  c->kstat[K_SWEEP_LAST].bytes = 4 * 18 * Nd * s + tmat + Nd + 5 * cons;
  TRY(build_rhs_tiles(c, m, halo_off, halo));
  return FELBM_OK;
}

// felbm_diag from a device reduction record (and, with a context, the solver
// state of that context)
void fill_diag(const felbm_ctx* c, const DiagRecord& r, double residual, felbm_diag* out) {
  std::memset(out, 0, sizeof(*out));
  out->step = r.step;
  out->mass = r.mass;
  out->mean_ke = r.mean_ke;
  out->max_u = r.max_u;
  out->band_ke = r.band_ke;
  out->band_nodes = r.band_nodes;
  out->nonfinite = r.nonfinite;
  out->solver_sweeps = c ? c->prm.solver_sweeps : 0;
  out->solver_residual = (c && c->residual_step >= 0) ? residual : -1.0;
  out->residual_step = c ? c->residual_step : -1;
}

}  // namespace

extern "C" {

const char* felbm_last_error(const felbm_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int felbm_create(const felbm_params* p, felbm_ctx** out) {
  g_create_error.clear();
  if (!p || !out) {
    g_create_error = "create: null argument";
    return FELBM_EINVAL;
  }
  *out = nullptr;
  auto bad = [](double v) { return !std::isfinite(v); };
  if (bad(p->sigma) || bad(p->xi) || bad(p->mobility) || bad(p->rho_l) || bad(p->rho_v) || bad(p->nu_l) ||
      bad(p->nu_v) || bad(p->dt) || p->xi <= 0 || p->sigma < 0 || p->mobility < 0 || p->rho_l <= 0 || p->rho_v <= 0 ||
      p->nu_l <= 0 || p->nu_v <= 0 || p->dt <= 0) {
    g_create_error = "create: parameters must be finite with xi, densities, viscosities, dt > 0 and sigma, mobility >= 0";
    return FELBM_EINVAL;
  }
  if (p->precision != FELBM_FP64 && p->precision != FELBM_FP32) {
    g_create_error = "create: precision must be FELBM_FP64 or FELBM_FP32";
    return FELBM_EINVAL;
  }
  if (p->kernels != FELBM_KERNELS_AUTO && p->kernels != FELBM_KERNELS_GLOBAL) {
    g_create_error = "create: kernels must be FELBM_KERNELS_AUTO or FELBM_KERNELS_GLOBAL";
    return FELBM_EINVAL;
  }
  if (p->force_scheme != FELBM_FORCES_MIXED && p->force_scheme != FELBM_FORCES_NODAL &&
      p->force_scheme != FELBM_FORCES_NODAL_COLLIDE) {
    g_create_error = "create: force_scheme must be FELBM_FORCES_MIXED, _NODAL or _NODAL_COLLIDE";
    return FELBM_EINVAL;
  }
  if (p->force_scheme != FELBM_FORCES_MIXED && p->precision != FELBM_FP64) {
    g_create_error = "create: the nodal force schemes are available in FP64 only";
    return FELBM_EINVAL;
  }
  if (p->solver_sweeps < 0 || p->solver_sweeps > 256) {
    g_create_error = "create: solver_sweeps must be in [0, 256]";
    return FELBM_EINVAL;
  }
  double lo = p->lambda_min, hi = p->lambda_max;
  if (lo == 0.0 && hi == 0.0) {
    lo = 0.25;
    hi = 1.0;
  }
  if (!(lo > 0.0 && hi > lo) || bad(lo) || bad(hi)) {
    g_create_error = "create: need 0 < lambda_min < lambda_max";
    return FELBM_EINVAL;
  }
  felbm_ctx* c = new (std::nothrow) felbm_ctx();
  if (!c) {
    g_create_error = "create: out of host memory";
    return FELBM_ENOMEM;
  }
  c->prm = *p;
  c->prm.lambda_min = lo;
  c->prm.lambda_max = hi;
  c->rs = p->precision == FELBM_FP64 ? 8 : 4;
  const double kappa = 1.5 * p->sigma * p->xi, beta = 12.0 * p->sigma / p->xi;  // xi = sqrt(8k/b), sigma = sqrt(2kb)/6
  c->sp = StepParams{kappa, beta, p->mobility, p->rho_l, p->rho_v, CS2 * p->dt / p->nu_l, CS2 * p->dt / p->nu_v, p->dt};
  c->cheb_w = chebyshev_steps(p->solver_sweeps, lo, hi);
  if (hipGetDevice(&c->device) != hipSuccess || hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
    g_create_error = "create: no usable HIP device";
    delete c;
    return FELBM_EDEVICE;
  }
  c->stream = c->own_stream;
  if (const int r = noalloc_scratch_for_current_device(c->device, &c->noalloc_scratch, g_create_error); r != FELBM_OK) {
    (void)hipStreamDestroy(c->own_stream);
    delete c;
    return r;
  }
  *out = c;
  return FELBM_OK;
}

int felbm_upload_mesh(felbm_ctx* c, int64_t n_nodes, const double* xy, int64_t n_tris, const int32_t* tri,
                      int64_t n_wall_edges, const int32_t* wall_edge, double period_x) {
  if (!c) return FELBM_EINVAL;
  if (c->has_mesh) return fail(c, FELBM_ESTATE, "upload_mesh: a mesh was already uploaded to this context");
  MeshPrep m;
  int r = prepare_mesh(n_nodes, xy, n_tris, tri, n_wall_edges, wall_edge, period_x, m, c->err);
  if (r != FELBM_OK) return r;
  c->N = m.N;
  c->Np = m.Np;
  c->E = m.E;
  c->W = m.W;
  c->offdiag_nnz = m.offdiag_nnz;
  c->node_perm = m.node_perm;
  c->elem_perm = m.elem_perm;
  c->perm_hash = m.perm_hash;
  c->sell_entries = (int64_t)m.sell_col.size();
  c->band.period = period_x;
  HIP_OK(c, hipSetDevice(c->device));
  const int64_t N = m.N, Np = m.Np, E = m.E;
  const size_t rs = c->rs;
  TRY(dalloc(c, &c->tri, 3 * E));
  TRY(dalloc(c, &c->enbr, 3 * E));
  TRY(dalloc(c, &c->geo, 7 * E));
  TRY(dalloc_bytes(c, &c->geor, 7 * E * rs));
  TRY(dalloc(c, &c->n2e_ptr, N + 1));
  TRY(dalloc(c, &c->n2e, 3 * E));
  TRY(dalloc(c, &c->wall_nbr, 2 * N));
  TRY(dalloc(c, &c->wall_len, 2 * N));
  TRY(dalloc(c, &c->is_wall, N));
  TRY(dalloc(c, &c->bc, N));
  TRY(dalloc(c, &c->mass, N));
  TRY(dalloc(c, &c->pvol, N));
  TRY(dalloc(c, &c->eflux, 3 * E));
  TRY(dalloc(c, &c->xy, 2 * N));
  TRY(dalloc(c, &c->sell_ptr, m.sell_ptr.size()));
  TRY(dalloc(c, &c->sell_col, m.sell_col.size()));
  TRY(dalloc_bytes(c, &c->sell_val, m.sell_val.size() * rs));
  TRY(dalloc_bytes(c, &c->pop, 18 * Np * rs));
  TRY(dalloc_bytes(c, &c->f, 18 * Np * rs));
  TRY(dalloc_bytes(c, &c->xa, 18 * Np * rs));
  TRY(dalloc_bytes(c, &c->xb, 18 * Np * rs));
  TRY(dalloc(c, &c->Cn, N));
  TRY(dalloc(c, &c->mu, N));
  TRY(dalloc(c, &c->lapC, N));
  TRY(dalloc_bytes(c, &c->pn, N * rs));
  TRY(dalloc_bytes(c, &c->uxn, N * rs));
  TRY(dalloc_bytes(c, &c->uyn, N * rs));
  TRY(dalloc(c, &c->gC, 2 * E));
  TRY(dalloc(c, &c->gmu, 2 * E));
  TRY(dalloc(c, &c->lapmu, E));
  TRY(dalloc_bytes(c, &c->gp, 2 * E * rs));
  if (c->prm.force_scheme == FELBM_FORCES_NODAL) TRY(dalloc_bytes(c, &c->Fn, 18 * Np * rs));
  if (c->prm.force_scheme == FELBM_FORCES_NODAL_COLLIDE) TRY(dalloc(c, &c->lapmu_n, N));
  if (c->prm.precision == FELBM_FP32) {
    TRY(dalloc(c, &c->rC, Np));
    TRY(dalloc(c, &c->fC, Np));
    TRY(dalloc(c, &c->xCa, Np));
    TRY(dalloc(c, &c->xCb, Np));
    TRY(dalloc(c, &c->dlt, Np));
  }
  TRY(dalloc(c, &c->partials, (size_t)NRED * grid_for(N)));
  TRY(dalloc(c, &c->res_partials, (size_t)NRES * grid_for(N)));
  TRY(dalloc(c, &c->res_out, 1));
  TRY(dalloc(c, &c->hist, c->hist_cap));
  TRY(dalloc(c, &c->diag_now, 1));
  TRY(dalloc(c, &c->first_bad, 1));
  TRY(upload(c, c->tri, m.tri));
  TRY(upload(c, c->enbr, m.enbr));
  TRY(upload(c, c->geo, m.geo));
  TRY(upload(c, c->n2e_ptr, m.n2e_ptr));
  TRY(upload(c, c->n2e, m.n2e));
  TRY(upload(c, c->wall_nbr, m.wall_nbr));
  TRY(upload(c, c->wall_len, m.wall_len));
  TRY(upload(c, c->is_wall, m.is_wall));
  TRY(upload(c, c->mass, m.mass));
  {
    // patch volume sum_T A_T in the node's element-list order (the order the gather sums its fluxes)
    std::vector<double> pvol(N, 0.0);
    for (int64_t k = 0; k < N; ++k)
      for (int32_t q = m.n2e_ptr[k]; q < m.n2e_ptr[k + 1]; ++q) pvol[k] += m.geo[m.n2e[q] >> 2];
    TRY(upload(c, c->pvol, pvol));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (c->prm.precision == FELBM_FP64)
      TRY(build_field_operators<double>(c, m, pvol));
    else
      TRY(build_field_operators<float>(c, m, pvol));
  }
  TRY(upload(c, c->xy, m.xy));
  TRY(upload(c, c->sell_ptr, m.sell_ptr));
  TRY(upload(c, c->sell_col, m.sell_col));
  if (c->prm.precision == FELBM_FP64) {
    TRY(upload(c, (double*)c->geor, m.geo));
    TRY(upload(c, (double*)c->sell_val, m.sell_val));
  } else {
    std::vector<float> g32(m.geo.begin(), m.geo.end()), v32(m.sell_val.begin(), m.sell_val.end());
    TRY(upload(c, (float*)c->geor, g32));
    TRY(upload(c, (float*)c->sell_val, v32));
    // diagonal of the FP64 composition sweep: dlt_j = 1 - sum_i m_i a_ij / m_j
    // with the stored (FP32) a_ij, so that m^T A = m^T exactly
    std::vector<double> colsum(Np, 0.0), dlt(Np, 0.5);
    const int64_t nslices = Np / 64;
    for (int64_t s = 0; s < nslices; ++s) {
      const int64_t base = m.sell_ptr[s], w = (m.sell_ptr[s + 1] - base) / 64;
      for (int lane = 0; lane < 64; ++lane) {
        const int64_t i = s * 64 + lane;
        if (i >= N) continue;
        for (int64_t k = 0; k < w; ++k) {
          const int64_t idx = base + k * 64 + lane;
          colsum[m.sell_col[idx]] += m.mass[i] * (double)v32[idx];
        }
      }
    }
    for (int64_t j = 0; j < N; ++j) dlt[j] = 1.0 - colsum[j] / m.mass[j];
    TRY(upload(c, c->dlt, dlt));
    HIP_OK(c, hipStreamSynchronize(c->stream));  // host vectors are about to go out of scope
  }
  {
    std::vector<int32_t> erev(3 * E, -1);
    for (int64_t e = 0; e < E; ++e)
      for (int l = 0; l < 3; ++l) {
        const int32_t nb = m.enbr[l * E + e];
        if (nb < 0) continue;
        for (int r = 0; r < 3; ++r)
          if (m.enbr[r * E + nb] == (int32_t)e) erev[l * E + e] = r;
      }
    TRY(dalloc(c, &c->erev, 3 * E));
    TRY(upload(c, c->erev, erev));
    TRY(dalloc(c, &c->d_node_perm, N));
    TRY(upload(c, c->d_node_perm, m.node_perm));
    TRY(dalloc(c, &c->wet_flags, 2));
    HIP_OK(c, hipStreamSynchronize(c->stream));
  }
  set_kernel_bytes(c);
  if (c->prm.kernels == FELBM_KERNELS_AUTO) TRY(build_tiles(c, m));
  std::vector<double> zeros(N, 0.0);
  TRY(upload(c, c->bc, zeros));
  HIP_OK(c, hipMemsetAsync(c->pop, 0, 18 * Np * rs, c->stream));
  HIP_OK(c, hipMemsetAsync(c->f, 0, 18 * Np * rs, c->stream));
  HIP_OK(c, hipMemsetAsync(c->xa, 0, 18 * Np * rs, c->stream));
  HIP_OK(c, hipMemsetAsync(c->xb, 0, 18 * Np * rs, c->stream));
  HIP_OK(c, hipMemsetAsync(c->hist, 0, c->hist_cap * sizeof(DiagRecord), c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->host_omega.assign(N, 0.0);
  c->has_mesh = true;
  return FELBM_OK;
}

int felbm_set_wetting(felbm_ctx* c, const double* omega_c) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_mesh) return fail(c, FELBM_ESTATE, "set_wetting: no mesh");
  if (!omega_c) return fail(c, FELBM_EINVAL, "set_wetting: null omega_c");
  const double kappa = c->sp.kappa, beta = c->sp.beta;
  std::vector<double> bc(c->N, 0.0);
  for (int64_t k = 0; k < c->N; ++k) {
    const double v = omega_c[c->node_perm[k]];
    if (!std::isfinite(v)) return fail(c, FELBM_EINVAL, "set_wetting: non-finite value");
    c->host_omega[k] = v;
  }
  // wall flags live on the device; recompute them from the host copy of the mesh is not kept, so read back
  std::vector<uint8_t> wall(c->N);
  HIP_OK(c, hipMemcpy(wall.data(), c->is_wall, c->N, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < c->N; ++i) {
    const double om = c->host_omega[i];
    if (!wall[i] || om == 0.0) continue;
    if (kappa <= 0.0) return fail(c, FELBM_EINVAL, "set_wetting: a nonzero wetting potential needs kappa > 0");
    bc[i] = om * std::sqrt(2.0 * kappa * beta) / kappa;  // phi_c / kappa, Young: phi_c = Omega_c sqrt(2 kappa beta)
  }
  invalidate_adjoint(c);
  TRY(upload(c, c->bc, bc));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return FELBM_OK;
}

int felbm_set_wetting_device(felbm_ctx* c, const double* omega_dev) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_mesh) return fail(c, FELBM_ESTATE, "set_wetting_device: no mesh");
  if (!omega_dev) return fail(c, FELBM_EINVAL, "set_wetting_device: null omega_c");
  const double kappa = c->sp.kappa, beta = c->sp.beta;
  const int N = (int)c->N, g1 = (N + BLOCK - 1) / BLOCK;
  // validate first, so that a rejected call leaves the wetting field as it was
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, c->wet_flags, 2, 0);
  hipLaunchKernelGGL(k_wetting_check, dim3(g1), dim3(BLOCK), 0, c->stream, N, (const int*)c->d_node_perm,
                     (const uint8_t*)c->is_wall, omega_dev, c->wet_flags);
  HIP_OK(c, hipGetLastError());
  int32_t flags[2] = {0, 0};
  HIP_OK(c, hipMemcpyAsync(flags, c->wet_flags, sizeof flags, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (flags[0]) return fail(c, FELBM_EINVAL, "set_wetting_device: non-finite value");
  if (flags[1] && kappa <= 0.0)
    return fail(c, FELBM_EINVAL, "set_wetting_device: a nonzero wetting potential needs kappa > 0");
  invalidate_adjoint(c);
  const double sq = flags[1] ? std::sqrt(2.0 * kappa * beta) : 0.0;
  hipLaunchKernelGGL(k_wetting_bc, dim3(g1), dim3(BLOCK), 0, c->stream, N, (const int*)c->d_node_perm,
                     (const uint8_t*)c->is_wall, omega_dev, sq, flags[1] ? kappa : 1.0, c->bc);
  HIP_OK(c, hipGetLastError());
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return FELBM_OK;
}

int felbm_init(felbm_ctx* c, const double* C, const double* u, const double* p) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_mesh) return fail(c, FELBM_ESTATE, "init: no mesh");
  if (!C) return fail(c, FELBM_EINVAL, "init: null C");
  const int64_t N = c->N;
  std::vector<double> hC(N), hU(2 * N, 0.0), hP(N, 0.0);
  for (int64_t k = 0; k < N; ++k) {
    const int64_t s = c->node_perm[k];
    hC[k] = C[s];
    if (u) {
      hU[2 * k] = u[2 * s];
      hU[2 * k + 1] = u[2 * s + 1];
    }
    if (p) hP[k] = p[s];
  }
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(hC[i]) || !std::isfinite(hU[2 * i]) || !std::isfinite(hU[2 * i + 1]) || !std::isfinite(hP[i]))
      return fail(c, FELBM_EINVAL, "init: non-finite input at node " + std::to_string(i));
  invalidate_adjoint(c);
  double *dC = nullptr, *dU = nullptr, *dP = nullptr;
  HIP_OK(c, hipMallocAsync((void**)&dC, N * 8, c->stream));
  HIP_OK(c, hipMallocAsync((void**)&dU, 2 * N * 8, c->stream));
  HIP_OK(c, hipMallocAsync((void**)&dP, N * 8, c->stream));
  HIP_OK(c, hipMemcpyAsync(dC, hC.data(), N * 8, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(dU, hU.data(), 2 * N * 8, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(dP, hP.data(), N * 8, hipMemcpyHostToDevice, c->stream));
  const int g = (int)((N + BLOCK - 1) / BLOCK);
  if (c->prm.precision == FELBM_FP64)
    hipLaunchKernelGGL(k_init<double>, dim3(g), dim3(BLOCK), 0, c->stream, (int)N, (int)c->Np, c->sp, (const double*)dC,
                       (const double*)dU, (const double*)dP, (const uint8_t*)c->is_wall, (double*)c->pop, c->rC);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(g), dim3(BLOCK), 0, c->stream, (int)N, (int)c->Np, c->sp, (const double*)dC,
                       (const double*)dU, (const double*)dP, (const uint8_t*)c->is_wall, (float*)c->pop, c->rC);
  HIP_OK(c, hipGetLastError());
  if (c->prm.force_scheme == FELBM_FORCES_NODAL_COLLIDE) TRY(enqueue_nc_init<double>(c));
  HIP_OK(c, hipFreeAsync(dC, c->stream));
  HIP_OK(c, hipFreeAsync(dU, c->stream));
  HIP_OK(c, hipFreeAsync(dP, c->stream));
  const int32_t minus1 = -1;
  HIP_OK(c, hipMemcpyAsync(c->first_bad, &minus1, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->step = 0;
  c->has_state = true;
  return FELBM_OK;
}

int felbm_step_async(felbm_ctx* c, int64_t n) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "step: not initialised");
  if (n < 0) return fail(c, FELBM_EINVAL, "step: negative step count");
  if (n > 0) invalidate_adjoint(c);
  return enqueue_steps(c, n);
}

int felbm_step(felbm_ctx* c, int64_t n) {
  TRY(felbm_step_async(c, n));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->timing) TRY(harvest_timing(c));
  int32_t bad = -1;
  HIP_OK(c, hipMemcpy(&bad, c->first_bad, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (bad >= 0) return fail(c, FELBM_ENONFINITE, "step: non-finite state entering step " + std::to_string(bad));
  return FELBM_OK;
}

int felbm_read(felbm_ctx* c, int32_t field, double* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "read: not initialised");
  if (!out) return fail(c, FELBM_EINVAL, "read: null output");
  if (field < FELBM_FIELD_C || field > FELBM_FIELD_LAPMU) return fail(c, FELBM_EINVAL, "read: unknown field");
  TRY(enqueue_fields_any(c, false, false, nullptr, read_field_mode(c)));
  const int64_t N = c->N;
  const double* src = nullptr;
  double* tmp = nullptr;
  int64_t n = N;
  switch (field) {
    case FELBM_FIELD_C:
    case FELBM_FIELD_RHO: src = c->Cn; break;
    case FELBM_FIELD_MU: src = c->mu; break;
    case FELBM_FIELD_LAPC: src = c->lapC; break;
    case FELBM_FIELD_LAPMU: src = c->lapmu; n = c->E; break;
    default: {
      const void* s = field == FELBM_FIELD_P ? c->pn : (field == FELBM_FIELD_UX ? c->uxn : c->uyn);
      HIP_OK(c, hipMallocAsync((void**)&tmp, N * 8, c->stream));
      TRY(to_double(c, s, tmp, N));
      src = tmp;
    }
  }
  std::vector<double> host(n);
  HIP_OK(c, hipMemcpyAsync(host.data(), src, n * 8, hipMemcpyDeviceToHost, c->stream));
  if (tmp) HIP_OK(c, hipFreeAsync(tmp, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->timing) TRY(harvest_timing(c));
  const std::vector<int32_t>& perm = field == FELBM_FIELD_LAPMU ? c->elem_perm : c->node_perm;
  for (int64_t k = 0; k < n; ++k) out[perm[k]] = host[k];
  if (field == FELBM_FIELD_RHO)
    for (int64_t i = 0; i < N; ++i) out[i] = out[i] * c->prm.rho_l + (1.0 - out[i]) * c->prm.rho_v;
  return FELBM_OK;
}

int felbm_read_device(felbm_ctx* c, int32_t field, double* out_dev) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "read_device: not initialised");
  if (!out_dev) return fail(c, FELBM_EINVAL, "read_device: null output");
  if (field < FELBM_FIELD_C || field > FELBM_FIELD_LAPC)
    return fail(c, FELBM_EINVAL, "read_device: not a nodal field (element fields: felbm_read)");
  TRY(enqueue_fields_any(c, false, false, nullptr, read_field_mode(c)));
  const int N = (int)c->N, g1 = (N + BLOCK - 1) / BLOCK;
  const double* src = nullptr;
  double* tmp = nullptr;
  switch (field) {
    case FELBM_FIELD_C:
    case FELBM_FIELD_RHO: src = c->Cn; break;
    case FELBM_FIELD_MU: src = c->mu; break;
    case FELBM_FIELD_LAPC: src = c->lapC; break;
    default: {
      const void* s = field == FELBM_FIELD_P ? c->pn : (field == FELBM_FIELD_UX ? c->uxn : c->uyn);
      HIP_OK(c, hipMallocAsync((void**)&tmp, (size_t)N * 8, c->stream));
      TRY(to_double(c, s, tmp, N));
      src = tmp;
    }
  }
  hipLaunchKernelGGL(k_field_to_caller, dim3(g1), dim3(BLOCK), 0, c->stream, N, (const int*)c->d_node_perm, src,
                     out_dev, field == FELBM_FIELD_RHO ? 1 : 0, c->prm.rho_l, c->prm.rho_v);
  HIP_OK(c, hipGetLastError());
  if (tmp) HIP_OK(c, hipFreeAsync(tmp, c->stream));
  return FELBM_OK;
}

int felbm_read_populations(felbm_ctx* c, double* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "read_populations: not initialised");
  if (!out) return fail(c, FELBM_EINVAL, "read_populations: null output");
  return copy_pops_out(c, c->pop, out);
}

int felbm_step_debug(felbm_ctx* c, double* psi_hat, double* rhs_over_m, double* delta) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "step_debug: not initialised");
  invalidate_adjoint(c);
  // the step's pipeline, split after the right-hand side to capture psi_hat and b/m
  TRY(enqueue_fields_any(c, true, true, c->hist + (c->step % c->hist_cap), step_field_mode(c)));
  if (c->prm.precision == FELBM_FP64)
    TRY(enqueue_rhs<double>(c));
  else
    TRY(enqueue_rhs<float>(c));
  std::vector<double> hat(18 * c->N);
  TRY(copy_pops_out(c, c->pop, hat.data()));
  if (psi_hat) std::memcpy(psi_hat, hat.data(), hat.size() * 8);
  if (rhs_over_m) TRY(copy_pops_out(c, c->f, rhs_over_m));
  if (c->prm.precision == FELBM_FP64)
    TRY(enqueue_solve<double>(c));
  else
    TRY(enqueue_solve<float>(c));
  c->step += 1;
  if (delta) {
    std::vector<double> after(18 * c->N);
    TRY(copy_pops_out(c, c->pop, after.data()));
    std::vector<uint8_t> wall_int(c->N), wall(c->N);
    HIP_OK(c, hipMemcpy(wall_int.data(), c->is_wall, c->N, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < c->N; ++k) wall[c->node_perm[k]] = wall_int[k];
    // delta = psi_bar^{n+1} - psi_hat at interior nodes; wall nodes get NaN
    // because the wall operator has already been applied there
    for (int64_t a = 0; a < 18; ++a)
      for (int64_t i = 0; i < c->N; ++i)
        delta[a * c->N + i] = wall[i] ? std::nan("") : after[a * c->N + i] - hat[a * c->N + i];
  }
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->timing) TRY(harvest_timing(c));
  return FELBM_OK;
}

int felbm_set_band(felbm_ctx* c, double xc, double yc, double R, double w) {
  if (!c) return FELBM_EINVAL;
  if (!std::isfinite(xc) || !std::isfinite(yc) || !std::isfinite(R) || !std::isfinite(w) || w < 0)
    return fail(c, FELBM_EINVAL, "set_band: bad arguments");
  if (R <= 0) {
    c->band.enabled = 0;
    return FELBM_OK;
  }
  const double lo = std::max(0.0, R - w), hi = R + w;
  c->band.xc = xc;
  c->band.yc = yc;
  c->band.r_lo2 = lo * lo;
  c->band.r_hi2 = hi * hi;
  c->band.enabled = 1;
  return FELBM_OK;
}

int felbm_diagnostics(felbm_ctx* c, felbm_diag* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "diagnostics: not initialised");
  if (!out) return fail(c, FELBM_EINVAL, "diagnostics: null output");

  const int gN = grid_for(c->N);
  const int N = (int)c->N, Np = (int)c->Np;
  int32_t* scratch_bad = nullptr;
  HIP_OK(c, hipMallocAsync((void**)&scratch_bad, sizeof(int32_t), c->stream));
  const int32_t zero = 0;
  HIP_OK(c, hipMemcpyAsync(scratch_bad, &zero, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  if (c->prm.force_scheme == FELBM_FORCES_NODAL_COLLIDE)
    // the velocity carries half the force's first moment: reduce the corrected fields
    TRY(enqueue_fields_any(c, false, false, nullptr, FIELDS_FULL));
  else if (c->prm.precision == FELBM_FP64)
    TRY(launch(c, K_MOMENTS, k_moments<double, false>, gN, (double*)c->pop, N, Np, c->sp, c->Cn, (double*)c->pn,
               (double*)c->uxn, (double*)c->uyn, (const double*)c->mass, (const double*)c->xy, c->band, (const double*)c->rC, c->partials));
  else
    TRY(launch(c, K_MOMENTS, k_moments<float, false>, gN, (float*)c->pop, N, Np, c->sp, c->Cn, (float*)c->pn,
               (float*)c->uxn, (float*)c->uyn, (const double*)c->mass, (const double*)c->xy, c->band, (const double*)c->rC, c->partials));
  TRY(launch_bs(c, K_REDUCE, k_reduce_final<>, 1, RBLOCK, (const double*)c->partials, gN, N, (int64_t)c->step, c->diag_now,
             scratch_bad));
  DiagRecord rec;
  double res = -1.0;
  HIP_OK(c, hipMemcpyAsync(&rec, c->diag_now, sizeof(DiagRecord), hipMemcpyDeviceToHost, c->stream));
  if (c->residual_step >= 0) HIP_OK(c, hipMemcpyAsync(&res, c->res_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipFreeAsync(scratch_bad, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->timing) TRY(harvest_timing(c));
  fill_diag(c, rec, res, out);
  return FELBM_OK;
}

int felbm_diagnostics_noalloc(felbm_ctx* c, felbm_diag* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "diagnostics_noalloc: not initialised");
  if (!out) return fail(c, FELBM_EINVAL, "diagnostics_noalloc: null output");
  if (c->prm.force_scheme == FELBM_FORCES_NODAL_COLLIDE)
    return fail(c, FELBM_EINVAL, "diagnostics_noalloc: not available for the collision-step nodal scheme");
  const int gN = grid_for(c->N);
  if (gN > kNoAllocMaxBlocks)
    return fail(c, FELBM_EINVAL, "diagnostics_noalloc: " + std::to_string(c->N) + " nodes exceed the no-alloc scratch (at most " +
                                     std::to_string((int64_t)kNoAllocMaxBlocks * BLOCK) + " nodes); use felbm_diagnostics");
  if (!c->noalloc_scratch) return fail(c, FELBM_EDEVICE, "diagnostics_noalloc: no scratch address for this device");
  const int N = (int)c->N, Np = (int)c->Np;
  double* partials = static_cast<double*>(c->noalloc_scratch);
  DiagRecord* rec = reinterpret_cast<DiagRecord*>(partials + kNoAllocRecordOffset);
  int32_t* flag = reinterpret_cast<int32_t*>(rec + 1);
  // the flag is written only where it is negative; 0 keeps it untouched (a
  // fill kernel, not a memset node, so that a captured call replays it)
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, flag, 1, 0);
  if (c->prm.precision == FELBM_FP64)
    hipLaunchKernelGGL((k_moments<double, false>), dim3(gN), dim3(BLOCK), 0, c->stream, (double*)c->pop, N, Np, c->sp,
                       c->Cn, (double*)c->pn, (double*)c->uxn, (double*)c->uyn, (const double*)c->mass,
                       (const double*)c->xy, c->band, (const double*)c->rC, partials);
  else
    hipLaunchKernelGGL((k_moments<float, false>), dim3(gN), dim3(BLOCK), 0, c->stream, (float*)c->pop, N, Np, c->sp,
                       c->Cn, (float*)c->pn, (float*)c->uxn, (float*)c->uyn, (const double*)c->mass,
                       (const double*)c->xy, c->band, (const double*)c->rC, partials);
  hipLaunchKernelGGL(k_reduce_final<>, dim3(1), dim3(RBLOCK), 0, c->stream, (const double*)partials, gN, N,
                     (int64_t)c->step, rec, flag);
  HIP_OK(c, hipGetLastError());
  DiagRecord host;
  double res = -1.0;
  HIP_OK(c, hipMemcpyAsync(&host, rec, sizeof(DiagRecord), hipMemcpyDeviceToHost, c->stream));
  if (c->residual_step >= 0) HIP_OK(c, hipMemcpyAsync(&res, c->res_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  fill_diag(c, host, res, out);
  return FELBM_OK;
}

int felbm_set_residual_sampling(felbm_ctx* c, int64_t every) {
  if (!c) return FELBM_EINVAL;
  if (every < 0) return fail(c, FELBM_EINVAL, "set_residual_sampling: negative interval");
  c->residual_every = every;
  return FELBM_OK;
}

int felbm_history(felbm_ctx* c, felbm_diag* out, int64_t max_entries, int64_t* n_out) {
  if (!c) return FELBM_EINVAL;
  if (!out || !n_out || max_entries < 0) return fail(c, FELBM_EINVAL, "history: bad arguments");
  HIP_OK(c, hipStreamSynchronize(c->stream));
  const int64_t avail = std::min<int64_t>(c->step, c->hist_cap);
  const int64_t n = std::min<int64_t>(avail, max_entries);
  std::vector<DiagRecord> all(c->hist_cap);
  if (n > 0) HIP_OK(c, hipMemcpy(all.data(), c->hist, c->hist_cap * sizeof(DiagRecord), hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < n; ++k) {
    const int64_t s = c->step - n + k;
    fill_diag(nullptr, all[s % c->hist_cap], -1.0, &out[k]);
  }
  *n_out = n;
  return FELBM_OK;
}

namespace {
int64_t payload_bytes(const felbm_ctx* c) {
  // populations in compute precision, plus the FP64 composition remainder in FP32 mode
  return 18 * c->Np * (int64_t)c->rs + (c->prm.precision == FELBM_FP32 ? c->Np * 8 : 0);
}
}  // namespace

int64_t felbm_state_bytes(const felbm_ctx* c) {
  if (!c || !c->has_mesh) return 0;
  return (int64_t)sizeof(StateHeader) + payload_bytes(c);
}

int felbm_save_state(felbm_ctx* c, void* buf, int64_t bytes) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "save_state: not initialised");
  if (!buf || bytes < felbm_state_bytes(c)) return fail(c, FELBM_EINVAL, "save_state: buffer too small");
  StateHeader h{kStateMagic, c->prm.precision, c->N, c->step, payload_bytes(c), c->perm_hash};
  std::memcpy(buf, &h, sizeof(h));
  const int64_t pb = 18 * c->Np * (int64_t)c->rs;
  HIP_OK(c, hipMemcpyAsync((char*)buf + sizeof(h), c->pop, pb, hipMemcpyDeviceToHost, c->stream));
  if (c->rC) HIP_OK(c, hipMemcpyAsync((char*)buf + sizeof(h) + pb, c->rC, c->Np * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return FELBM_OK;
}

int felbm_load_state(felbm_ctx* c, const void* buf, int64_t bytes) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_mesh) return fail(c, FELBM_ESTATE, "load_state: no mesh");
  if (!buf || bytes < felbm_state_bytes(c)) return fail(c, FELBM_EINVAL, "load_state: buffer too small");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kStateMagic || h.precision != c->prm.precision || h.n_nodes != c->N ||
      h.payload_bytes != payload_bytes(c) || h.perm_hash != c->perm_hash)
    return fail(c, FELBM_EINVAL, "load_state: header does not match this context");
  invalidate_adjoint(c);
  const int64_t pb = 18 * c->Np * (int64_t)c->rs;
  HIP_OK(c, hipMemcpyAsync(c->pop, (const char*)buf + sizeof(h), pb, hipMemcpyHostToDevice, c->stream));
  if (c->rC) HIP_OK(c, hipMemcpyAsync(c->rC, (const char*)buf + sizeof(h) + pb, c->Np * 8, hipMemcpyHostToDevice, c->stream));
  const int32_t minus1 = -1;
  HIP_OK(c, hipMemcpyAsync(c->first_bad, &minus1, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->step = h.step;
  c->has_state = true;
  return FELBM_OK;
}

int felbm_bind_stream(felbm_ctx* c, void* s) {
  if (!c) return FELBM_EINVAL;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->stream = s ? (hipStream_t)s : c->own_stream;
  return FELBM_OK;
}

int felbm_kernel_timing(felbm_ctx* c, int32_t enable) {
  if (!c) return FELBM_EINVAL;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  TRY(harvest_timing(c));
  c->timing = enable != 0;
  for (auto& k : c->kstat) {
    k.launches = 0;
    k.total_ms = 0.0;
  }
  return FELBM_OK;
}

int felbm_kernel_stats(felbm_ctx* c, felbm_kstat* out, int32_t max_entries, int32_t* n_out) {
  if (!c) return FELBM_EINVAL;
  if (!out || !n_out || max_entries < 0) return fail(c, FELBM_EINVAL, "kernel_stats: bad arguments");
  HIP_OK(c, hipStreamSynchronize(c->stream));
  TRY(harvest_timing(c));
  int n = std::min<int>(K_COUNT, max_entries);
  for (int k = 0; k < n; ++k) {
    std::memset(&out[k], 0, sizeof(felbm_kstat));
    std::snprintf(out[k].name, sizeof(out[k].name), "%s", kKernelNames[k]);
    out[k].launches = c->kstat[k].launches;
    out[k].total_ms = c->kstat[k].total_ms;
    out[k].bytes_per_launch = c->kstat[k].bytes;
  }
  *n_out = n;
  return FELBM_OK;
}

int felbm_forward_ckpt(felbm_ctx* c, int64_t n_steps, int64_t every) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "forward_ckpt: not initialised");
  if (n_steps < 1 || every < 1) return fail(c, FELBM_EINVAL, "forward_ckpt: n_steps and every must be >= 1");
  if (c->prm.force_scheme != FELBM_FORCES_MIXED)
    return fail(c, FELBM_EINVAL, "forward_ckpt: the adjoint covers the mixed force scheme only");
  invalidate_adjoint(c);
  TRY(ensure_adjoint_buffers(c));
  const size_t sb = dev_state_bytes(c);
  const int64_t nck = (n_steps + every - 1) / every;
  const size_t need_ck = (size_t)nck * sb, need_seg = (size_t)std::min(every, n_steps) * sb;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (need_ck > c->ck_cap) {
    if (c->ck_buf) HIP_OK(c, hipFree(c->ck_buf));
    c->ck_buf = nullptr;
    c->ck_cap = 0;
    if (hipMalloc(&c->ck_buf, need_ck) != hipSuccess) return fail(c, FELBM_ENOMEM, "forward_ckpt: checkpoint storage");
    c->ck_cap = need_ck;
  }
  if (need_seg > c->seg_cap) {
    if (c->seg_buf) HIP_OK(c, hipFree(c->seg_buf));
    c->seg_buf = nullptr;
    c->seg_cap = 0;
    if (hipMalloc(&c->seg_buf, need_seg) != hipSuccess) return fail(c, FELBM_ENOMEM, "forward_ckpt: segment storage");
    c->seg_cap = need_seg;
  }
  c->ck_every = every;
  c->ck_count = nck;
  c->ck_start = c->step;
  for (int64_t s = 0; s < n_steps; ++s) {
    if (s % every == 0) TRY(state_to(c, (char*)c->ck_buf + (size_t)(s / every) * sb));
    TRY(enqueue_steps(c, 1));
  }
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->timing) TRY(harvest_timing(c));
  int32_t bad = -1;
  HIP_OK(c, hipMemcpy(&bad, c->first_bad, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (bad >= 0) return fail(c, FELBM_ENONFINITE, "forward_ckpt: non-finite state entering step " + std::to_string(bad));
  // the checkpoints are complete: this run can be reversed
  c->ck_steps = n_steps;
  c->ck_run = ++c->ck_next_run;
  return FELBM_OK;
}

int felbm_adjoint_run(const felbm_ctx* c, int64_t* run_id) {
  if (!c || !run_id) return FELBM_EINVAL;
  *run_id = c->ck_steps > 0 ? c->ck_run : 0;
  return FELBM_OK;
}

namespace {
// the reverse sweep over all segments, from the seed already in c->lam
int backward_segments(felbm_ctx* c, double* dL_domega_dev) {
  const size_t sb = dev_state_bytes(c);
  const int N = (int)c->N;
  const int g1 = (N + BLOCK - 1) / BLOCK;
  HIP_OK(c, hipMemsetAsync(c->gomega, 0, c->Np * 8, c->stream));
  for (int64_t seg = c->ck_count - 1; seg >= 0; --seg) {
    const int64_t m0 = seg * c->ck_every, m1 = std::min(c->ck_steps, m0 + c->ck_every);
    // replay the segment, keeping every state
    TRY(state_from(c, (const char*)c->ck_buf + (size_t)seg * sb));
    c->step = c->ck_start + m0;
    for (int64_t m = m0; m < m1; ++m) {
      TRY(state_to(c, (char*)c->seg_buf + (size_t)(m - m0) * sb));
      if (m + 1 < m1) TRY(enqueue_steps(c, 1));
    }
    for (int64_t m = m1 - 1; m >= m0; --m) {
      TRY(state_from(c, (const char*)c->seg_buf + (size_t)(m - m0) * sb));
      TRY(enqueue_fields_any(c, false, false, nullptr, FIELDS_FULL));
      TRY(enqueue_adjoint_step_any(c));
    }
  }
  hipLaunchKernelGGL(k_to_caller, dim3(g1), dim3(BLOCK), 0, c->stream, N, (const int*)c->d_node_perm,
                     (const double*)c->gomega, dL_domega_dev);
  HIP_OK(c, hipGetLastError());
  return FELBM_OK;
}

// Reverse the last forward_ckpt run.  The replay overwrites the state, so the
// forward's final state and step counter are saved first and restored on
// every exit path; the saved copy is freed on every path as well.  If even
// the restoration fails, the context is marked as holding no state.
int run_backward(felbm_ctx* c, double* dL_domega_dev) {
  const size_t sb = dev_state_bytes(c);
  void* final_state = nullptr;
  HIP_OK(c, hipMallocAsync(&final_state, sb, c->stream));
  const int64_t end_step = c->step;
  int r = state_to(c, final_state);
  if (r == FELBM_OK) {
    r = backward_segments(c, dL_domega_dev);
    const std::string err = c->err;
    const int rr = state_from(c, final_state);
    c->step = end_step;
    if (rr != FELBM_OK) {
      c->has_state = false;
      invalidate_adjoint(c);
      if (r == FELBM_OK) r = rr;
    } else if (r != FELBM_OK) {
      c->err = err;  // report the first failure
    }
  }
  (void)hipFreeAsync(final_state, c->stream);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (r == FELBM_OK && e != hipSuccess) r = fail(c, FELBM_EDEVICE, std::string("backward: ") + hipGetErrorString(e));
  if (r == FELBM_OK && c->timing) r = harvest_timing(c);
  return r;
}
}  // namespace

int felbm_backward(felbm_ctx* c, const double* dL_dC_dev, double* dL_domega_dev) {
  if (!c) return FELBM_EINVAL;
  if (c->ck_steps <= 0) return fail(c, FELBM_ESTATE, "backward: no felbm_forward_ckpt run to reverse");
  if (!dL_dC_dev || !dL_domega_dev) return fail(c, FELBM_EINVAL, "backward: null device pointer");
  const int N = (int)c->N, Np = (int)c->Np;
  const int g1 = (N + BLOCK - 1) / BLOCK;
  if (c->prm.precision == FELBM_FP64)
    hipLaunchKernelGGL(k_adj_init<double>, dim3(g1), dim3(BLOCK), 0, c->stream, N, Np, (const int*)c->d_node_perm,
                       dL_dC_dev, (double*)c->lam);
  else
    hipLaunchKernelGGL(k_adj_init<float>, dim3(g1), dim3(BLOCK), 0, c->stream, N, Np, (const int*)c->d_node_perm,
                       dL_dC_dev, (float*)c->lam);
  HIP_OK(c, hipGetLastError());
  return run_backward(c, dL_domega_dev);
}

int felbm_backward_full(felbm_ctx* c, const double* dL_dpsi, const double* dL_dC, double* dL_domega,
                        double* dL_dpsi0) {
  if (!c) return FELBM_EINVAL;
  if (c->ck_steps <= 0) return fail(c, FELBM_ESTATE, "backward_full: no felbm_forward_ckpt run to reverse");
  if (!dL_domega) return fail(c, FELBM_EINVAL, "backward_full: null dL_domega");
  const int64_t N = c->N, Np = c->Np;
  std::vector<double> seed(18 * Np, 0.0);
  for (int64_t k = 0; k < N; ++k) {
    const int64_t s = c->node_perm[k];
    for (int a = 0; a < 18; ++a) {
      double v = dL_dpsi ? dL_dpsi[a * N + s] : 0.0;
      if (dL_dC && a >= 9) v += dL_dC[s];
      seed[a * Np + k] = v;
    }
  }
  if (c->prm.precision == FELBM_FP64) {
    HIP_OK(c, hipMemcpyAsync(c->lam, seed.data(), seed.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
  } else {
    std::vector<float> s32(seed.begin(), seed.end());
    HIP_OK(c, hipMemcpyAsync(c->lam, s32.data(), s32.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
  }
  double* dout = nullptr;
  HIP_OK(c, hipMalloc((void**)&dout, N * 8));
  int r = run_backward(c, dout);
  if (r == FELBM_OK && hipMemcpy(dL_domega, dout, N * 8, hipMemcpyDeviceToHost) != hipSuccess)
    r = fail(c, FELBM_EDEVICE, "backward_full: copy out");
  (void)hipFree(dout);
  if (r == FELBM_OK && dL_dpsi0) r = copy_pops_out(c, c->lam, dL_dpsi0);
  return r;
}

int felbm_backward_host(felbm_ctx* c, const double* dL_dC, double* dL_domega) {
  if (!c) return FELBM_EINVAL;
  if (!dL_dC || !dL_domega) return fail(c, FELBM_EINVAL, "backward_host: null pointer");
  double *din = nullptr, *dout = nullptr;
  HIP_OK(c, hipMalloc((void**)&din, c->N * 8));
  if (hipMalloc((void**)&dout, c->N * 8) != hipSuccess) {
    (void)hipFree(din);
    return fail(c, FELBM_ENOMEM, "backward_host: allocation");
  }
  int r = FELBM_OK;
  if (hipMemcpy(din, dL_dC, c->N * 8, hipMemcpyHostToDevice) != hipSuccess) r = fail(c, FELBM_EDEVICE, "copy in");
  if (r == FELBM_OK) r = felbm_backward(c, din, dout);
  if (r == FELBM_OK && hipMemcpy(dL_domega, dout, c->N * 8, hipMemcpyDeviceToHost) != hipSuccess)
    r = fail(c, FELBM_EDEVICE, "copy out");
  (void)hipFree(din);
  (void)hipFree(dout);
  return r;
}

int felbm_lumped_mass(felbm_ctx* c, double* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_mesh) return fail(c, FELBM_ESTATE, "lumped_mass: no mesh");
  if (!out) return fail(c, FELBM_EINVAL, "lumped_mass: null output");
  std::vector<double> m(c->N);
  HIP_OK(c, hipMemcpy(m.data(), c->mass, c->N * 8, hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < c->N; ++k) out[c->node_perm[k]] = m[k];
  return FELBM_OK;
}

int felbm_mesh_info(const felbm_ctx* c, int64_t* n_nodes, int64_t* n_tris, int64_t* n_wall_edges, int64_t* nnz) {
  if (!c || !c->has_mesh) return FELBM_ESTATE;
  if (n_nodes) *n_nodes = c->N;
  if (n_tris) *n_tris = c->E;
  if (n_wall_edges) *n_wall_edges = c->W;
  if (nnz) *nnz = c->offdiag_nnz;
  return FELBM_OK;
}

int felbm_validate_mesh(int64_t n_nodes, const double* xy, int64_t n_tris, const int32_t* tri, int64_t n_wall,
                        const int32_t* wall_edge, double period_x, char* msg, int32_t msg_len) {
  MeshPrep m;
  std::string err;
  const int r = prepare_mesh(n_nodes, xy, n_tris, tri, n_wall, wall_edge, period_x, m, err, false);
  if (msg && msg_len > 0) std::snprintf(msg, (size_t)msg_len, "%s", err.c_str());
  return r;
}

void felbm_destroy(felbm_ctx* c) {
  if (!c) return;
  // teardown: errors are not reportable past this point
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  for (void* p : c->allocations) (void)hipFree(p);
  if (c->ck_buf) (void)hipFree(c->ck_buf);
  if (c->seg_buf) (void)hipFree(c->seg_buf);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

}  // extern "C"
