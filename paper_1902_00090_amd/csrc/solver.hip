// Batched data-driven GMRES: workspace, augmentation setup and the cycle
// loop (Sec. 2, Eqs. 2-5; supplement Sec. 1).  Kernels are in
// solver_kernels.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "solver_kernels.h"
#include "solver_state.h"


// Fill the preconditioner arrays of every problem from its bound operator.
static hipError_t precond_init(dd_solver* s) {
  if (s->o.precond == DD_PRECOND_NONE) return hipSuccess;
  for (int p = 0; p < s->nb; ++p) {
    const auto& b = s->pcbuf[p];
    const int gx = std::min(256, (s->hdesc[p].Dp + DD_BLOCK - 1) / DD_BLOCK);
    k_precond_init<<<gx, DD_BLOCK>>>(s->P, p, s->o.precond, s->ops[p]->s64, b.pl64, b.pr64,
                                     b.pl32, b.pr32);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e;
}

extern "C" void dd_solver_opts_default(dd_solver_opts* o) {
  if (!o) return;
  o->inner = DD_C64;
  o->cgs_passes = 2;
  o->restart = 100;
  o->kmax = 0;
  o->elems_per_thread = 0;
  o->hist_cap = 0;
  o->check_every = 4;
  o->select_reorth = 1;
  o->use_graph = 0;
  o->precond = DD_PRECOND_NONE;
  o->workspace = nullptr;
  o->workspace_bytes = 0;
  o->fused = 0;
}

static size_t inner_bytes(dd_prec p) { return p == DD_C128 ? 16 : 8; }

// Device workspace layout: every array of a solver is carved, 256-byte
// aligned, from one block in a fixed order.  A first pass with base == NULL
// only measures the block (gmres_workspace_bytes); the second assigns the
// pointers into the solver's own allocation or the caller's workspace.
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename X>
  void carve(X** ptr, size_t count) {
    const size_t b = std::max<size_t>(count * sizeof(X), 256);
    off = (off + 255) & ~(size_t)255;
    *ptr = base ? (X*)(base + off) : nullptr;
    off += b;
  }
};

static void fill_desc_op(ProbDesc& d, const fdfd_op* op) {
  d.nx = op->nx;
  d.ny = op->ny;
  d.D = op->D;
  d.omega2 = op->omega * op->omega;
  d.eps32 = op->eps32;
  d.eps64 = op->eps64;
  d.cf32 = op->cf32;
  d.cf64 = op->cf64;
}

extern "C" void dd_solver_destroy(dd_solver* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->pinned) (void)hipHostFree(s->pinned);
  if (s->pinnedD) (void)hipHostFree(s->pinnedD);
  if (s->pinnedK) (void)hipHostFree(s->pinnedK);
  for (auto& e : s->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : s->pev)
    if (e) (void)hipEventDestroy(e);
  for (auto& g : s->execs)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& g : s->graphs)
    if (g) (void)hipGraphDestroy(g);
  if (s->cap) (void)hipStreamDestroy(s->cap);
  if (s->hctl) (void)hipHostFree(s->hctl);
  delete s;
}

// The arrays of a solver, in layout order (see Arena).
static void layout_workspace(dd_solver* s, Arena& A, ProbDesc*& dd, int*& db2p) {
  const dd_solver_opts& o = s->o;
  const int nb = s->nb, m = o.restart, K = o.kmax;
  const size_t ib = inner_bytes(o.inner);
  PlanDev& P = s->P;
  s->pcbuf.clear();
  for (int p = 0; p < nb; ++p) {
    ProbDesc& d = s->hdesc[p];
    char* basis = nullptr;
    char* V = nullptr;
    A.carve(&basis, (size_t)(K + m + 1) * d.Dp * ib);
    if (K > 0) A.carve(&V, (size_t)K * d.Dp * ib);
    double2* r = nullptr;
    A.carve(&r, (size_t)d.Dp);
    d.basis = basis;
    d.V = V;
    d.r = r;
    if (s->fused) {
      char* Z = nullptr;
      A.carve(&Z, (size_t)2 * d.Dp * ib);
      d.Z = Z;
    }
    if (o.precond != DD_PRECOND_NONE) {
      double2 *pl64 = nullptr, *pr64 = nullptr;
      float2 *pl32 = nullptr, *pr32 = nullptr;
      A.carve(&pl64, (size_t)d.Dp);
      A.carve(&pr64, (size_t)d.Dp);
      A.carve(&pl32, (size_t)d.Dp);
      A.carve(&pr32, (size_t)d.Dp);
      d.pl64 = pl64;
      d.pr64 = (o.precond == DD_PRECOND_PML) ? pr64 : nullptr;
      d.pl = (o.inner == DD_C64) ? (const void*)pl32 : (const void*)pl64;
      d.pr = (o.precond == DD_PRECOND_PML)
                 ? ((o.inner == DD_C64) ? (const void*)pr32 : (const void*)pr64) : nullptr;
      s->pcbuf.push_back({pl64, pr64, pl32, pr32});
    }
  }
  A.carve(&dd, nb);
  A.carve(&db2p, s->nchunks);
  if (s->fused) A.carve(&s->dtiles, s->htiles.size());
  A.carve(&s->dU, nb);
  A.carve(&P.stI, (size_t)nb * ST_NI);
  A.carve(&P.stD, (size_t)nb * SD_ND);
  A.carve(&P.H, (size_t)nb * m * (m + 1));
  A.carve(&P.Hraw, (size_t)nb * m * (m + 1));
  A.carve(&P.Bc, (size_t)nb * m * std::max(K, 1));
  A.carve(&P.g, (size_t)nb * (m + 1));
  A.carve(&P.cs, (size_t)nb * m);
  A.carve(&P.sn, (size_t)nb * m);
  A.carve(&P.c0, (size_t)nb * std::max(K, 1));
  A.carve(&P.coefA, (size_t)nb * P.NC);
  A.carve(&P.coefB, (size_t)nb * P.NC);
  A.carve(&P.coefA2, (size_t)nb * P.NC);
  A.carve(&P.hscale, (size_t)nb * (m + 1));
  A.carve(&P.comb, (size_t)nb * (K + m));
  A.carve(&P.Rinv, (size_t)nb * std::max(K * K, 1));
  A.carve(&P.Tm, (size_t)nb * std::max(K * K, 1));
  A.carve(&P.Gm, (size_t)nb * std::max(K * K, 1));
  A.carve(&P.keep, (size_t)nb);
  A.carve(&P.bad, (size_t)nb);
  double* part = nullptr;
  A.carve(&part, (size_t)std::max<size_t>(s->nchunks, s->htiles.size()) * P.NV);
  P.partial = part;
  A.carve(&P.gpart, (size_t)nb * P.GB * std::max(1, gram_tiles(std::max(K, 1))) * 32);
  A.carve(&P.hist, (size_t)nb * std::max(1, o.hist_cap));
  A.carve(&s->dctl, 2);
}

// Validates the options and builds the host-side plan of a solver (problem
// descriptors, chunk map, workspace parameters); no device memory yet.
extern "C" dd_status dd_solver_autotune(const fdfd_op* const* ops, int nb, const dd_solver_opts* opts,
                                        int* best, double* ms_per_step);

// elems_per_thread = -1: the autotuner's choice for this set of grid sizes and
// options, measured once per process and remembered.
static dd_status tuned_elems_per_thread(const fdfd_op* const* ops, int nb, const dd_solver_opts& o,
                                        int* R) {
  static std::mutex mu;
  static std::map<std::string, int> cache;
  std::string key = std::to_string(nb) + "/" + std::to_string(o.restart) + "/" +
                    std::to_string(o.inner) + "/" + std::to_string(o.cgs_passes) + "/" +
                    std::to_string(o.precond) + "/" + std::to_string(o.fused) + ":";
  for (int p = 0; p < nb; ++p) key += std::to_string(ops[p]->nx) + "x" + std::to_string(ops[p]->ny) + ",";
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) { *R = it->second; return DD_OK; }
  }
  dd_solver_opts t = o;
  t.elems_per_thread = 0;
  int best = 0;
  dd_status rc = dd_solver_autotune(ops, nb, &t, &best, nullptr);
  if (rc != DD_OK) return rc;
  std::lock_guard<std::mutex> lock(mu);
  cache[key] = best;
  *R = best;
  return DD_OK;
}

static dd_status solver_plan(const fdfd_op* const* ops, int nb, const dd_solver_opts* opts,
                             dd_solver** out) {
  if (!out) { dd_set_error("dd_solver_create: out is NULL"); return DD_EINVAL; }
  *out = nullptr;
  dd_solver_opts o;
  dd_solver_opts_default(&o);
  if (opts) o = *opts;
  if (o.check_every <= 0) o.check_every = 4;
  if (!ops || nb < 1) { dd_set_error("dd_solver_create: need nb >= 1 operators"); return DD_EINVAL; }
  for (int p = 0; p < nb; ++p)
    if (!ops[p]) { dd_set_error("dd_solver_create: ops[%d] is NULL", p); return DD_EINVAL; }
  if (o.restart < 1 || o.restart > DD_MAX_M) {
    dd_set_error("dd_solver_create: restart must be in 1..%d", DD_MAX_M);
    return DD_EINVAL;
  }
  if (o.kmax < 0 || o.kmax > DD_MAX_K) {
    dd_set_error("dd_solver_create: kmax must be in 0..%d", DD_MAX_K);
    return DD_EINVAL;
  }
  if (o.cgs_passes != 1 && o.cgs_passes != 2) {
    dd_set_error("dd_solver_create: cgs_passes must be 1 or 2");
    return DD_EINVAL;
  }
  if (o.inner != DD_C64 && o.inner != DD_C128) {
    dd_set_error("dd_solver_create: unknown inner precision");
    return DD_EINVAL;
  }
  if (o.hist_cap < 0) o.hist_cap = 0;
  if (o.precond != DD_PRECOND_NONE && o.precond != DD_PRECOND_JACOBI &&
      o.precond != DD_PRECOND_PML) {
    dd_set_error("dd_solver_create: unknown preconditioner %d", o.precond);
    return DD_EINVAL;
  }
  int R = o.elems_per_thread;
  if (R != -1 && R != 0 && R != 1 && R != 2 && R != 4 && R != 8) {
    dd_set_error("dd_solver_create: elems_per_thread must be -1, 0, 1, 2, 4 or 8");
    return DD_EINVAL;
  }
  if (R == -1) {
    dd_status rc = tuned_elems_per_thread(ops, nb, o, &R);
    if (rc != DD_OK) return rc;
  }
  if (R == 0) {
    // Measured by dd_solver_autotune on MI355X over full GMRES(100) cycles of
    // 480 x 240 problems: one problem is fastest with 2 elements per thread
    // (60 us/step against 63-77 for 1, 4 and 8); a batch of 64 takes 1.13-1.15
    // ms/step with 2, 4 or 8 against 1.35 with 1.  Large batches take 8 (the
    // fewest partial rows per problem), small ones 2.
    long long nch8 = 0;
    for (int p = 0; p < nb; ++p) nch8 += (ops[p]->D + DD_BLOCK * 8 - 1) / (DD_BLOCK * 8);
    R = (nch8 >= 512) ? 8 : 2;
  }
  dd_solver* s = new dd_solver();
  s->nb = nb;
  s->o = o;
  s->R = R;
  s->ops.assign(ops, ops + nb);
  s->hdesc.resize(nb);
  s->ksetup.assign(nb, 0);
  const int m = o.restart, K = o.kmax;
  const int chunk = DD_BLOCK * R;
  int blk = 0;
  for (int p = 0; p < nb; ++p) {
    ProbDesc& d = s->hdesc[p];
    std::memset(&d, 0, sizeof(d));
    fill_desc_op(d, ops[p]);
    d.nblk = (d.D + chunk - 1) / chunk;
    d.blk0 = blk;
    d.Dp = d.nblk * chunk;
    d.k = 0;
    blk += d.nblk;
  }
  s->nchunks = blk;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0)
      s->ncu = ncu;
  }
  const int NC = K + m + 1;
  const int NV = ((2 * NC + 31) / 32) * 32 + 32;
  PlanDev& P = s->P;
  P.nb = nb; P.m = m; P.kmax = K; P.NC = NC; P.NV = NV; P.hist_cap = o.hist_cap;
  P.qslots = m + 1;
  P.reorth_mode = (o.cgs_passes == 1) ? 0 : (o.select_reorth ? 2 : 1);
  // Gram partial rows: bounded to 64 MB
  {
    const size_t per = (size_t)nb * std::max(1, gram_tiles(std::max(K, 1))) * 32 * sizeof(double);
    int GB = (int)std::min<size_t>(32, std::max<size_t>(1, (64ull << 20) / per));
    P.GB = GB;
  }
  // Fused sweep tiles: strips of DD_FUSED_SW columns walked down bands of rows
  s->fused = o.fused && o.cgs_passes == 1 && (K + m + 1) <= DD_FUSED_MAXN;
  if (s->fused) {
    // two rounds of tiles over the resident workgroups (w per compute unit),
    // bands of 8 to 64 rows (each band recomputes one halo row at either end)
    int w = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &w, (o.inner == DD_C64) ? (const void*)k_fused_sweep<float, false>
                                    : (const void*)k_fused_sweep<double, false>,
            DD_FUSED_THREADS, 0) != hipSuccess || w < 1)
      w = 1;
    long long strip_rows = 0;
    for (int p = 0; p < nb; ++p)
      strip_rows += (long long)((ops[p]->nx + DD_FUSED_SW - 1) / DD_FUSED_SW) * ops[p]->ny;
    const long long slots = 2LL * w * s->ncu;
    const long long per = (strip_rows + slots - 1) / slots;
    const int bh = (int)std::min<long long>(64, std::max<long long>(8, per));
    std::vector<FusedTile> logical;
    for (int p = 0; p < nb; ++p) {
      ProbDesc& d = s->hdesc[p];
      const int nxp = ops[p]->nx, nyp = ops[p]->ny;
      d.t0 = (int)logical.size();
      for (int y0 = 0; y0 < nyp; y0 += bh)
        for (int x0 = 0; x0 < nxp; x0 += DD_FUSED_SW)
          logical.push_back({p, x0, y0, std::min(nyp, y0 + bh), 1, (int)logical.size()});
      d.nt = (int)logical.size() - d.t0;
    }
    // XCD-aware launch order: workgroup b runs on XCD b % 8, so XCD x is given
    // the x-th contiguous eighth of the tiles; neighbouring strips of a band
    // then share an L2, which serves the cache lines at their common edge
    const int X = 8;
    const int perx = (int)((logical.size() + X - 1) / X);
    s->htiles.assign((size_t)perx * X, FusedTile{-1, 0, 0, 0, 1, 0});
    for (int b = 0; b < perx * X; ++b) {
      const int i = (b % X) * perx + b / X;
      if (i < (int)logical.size()) s->htiles[b] = logical[i];
    }
  }
  *out = s;
  return DD_OK;
}

extern "C" dd_status dd_solver_create(const fdfd_op* const* ops, int nb, const dd_solver_opts* opts,
                                      dd_solver** out) {
  if (!out) { dd_set_error("dd_solver_create: out is NULL"); return DD_EINVAL; }
  *out = nullptr;
  dd_solver* s = nullptr;
  dd_status rc = solver_plan(ops, nb, opts, &s);
  if (rc != DD_OK) return rc;
  const dd_solver_opts& o = s->o;
  PlanDev& P = s->P;
  ProbDesc* dd = nullptr;
  int* db2p = nullptr;
  Arena A;
  layout_workspace(s, A, dd, db2p);
  const size_t total = A.off;
  hipError_t e = hipSuccess;
  if (o.workspace) {
    if (o.workspace_bytes < total || ((uintptr_t)o.workspace & 255) != 0) {
      dd_set_error("dd_solver_create: the workspace needs %zu bytes at 256-byte alignment "
                   "(got %zu bytes at %p)", total, o.workspace_bytes, o.workspace);
      delete s;
      return DD_EINVAL;
    }
    A.base = (char*)o.workspace;
    s->owns_workspace = false;
  } else {
    e = hipMalloc((void**)&A.base, total);
    if (e == hipSuccess) s->allocs.push_back(A.base);
  }
  if (e == hipSuccess) {
    s->bytes = total;
    A.off = 0;
    layout_workspace(s, A, dd, db2p);
    e = hipMemset(A.base, 0, total);
  }
  std::vector<int> b2p(s->nchunks);
  for (int p = 0; p < nb; ++p)
    for (int c = 0; c < s->hdesc[p].nblk; ++c) b2p[s->hdesc[p].blk0 + c] = p;
  auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  if (e == hipSuccess) {
    if (s->fused)
      chk(hipMemcpy(s->dtiles, s->htiles.data(), sizeof(FusedTile) * s->htiles.size(),
                    hipMemcpyHostToDevice));
    chk(hipMemcpy(dd, s->hdesc.data(), sizeof(ProbDesc) * nb, hipMemcpyHostToDevice));
    chk(hipMemcpy(db2p, b2p.data(), sizeof(int) * s->nchunks, hipMemcpyHostToDevice));
    chk(hipHostMalloc((void**)&s->pinned, sizeof(int) * 3 * nb * ST_NI, hipHostMallocDefault));
    chk(hipHostMalloc((void**)&s->pinnedD, sizeof(double) * nb * SD_ND, hipHostMallocDefault));
    chk(hipHostMalloc((void**)&s->pinnedK, sizeof(unsigned long long) * nb, hipHostMallocDefault));
    chk(hipHostMalloc((void**)&s->hctl, sizeof(double) * 2, hipHostMallocDefault));
    chk(hipEventCreateWithFlags(&s->ev[0], hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&s->ev[1], hipEventDisableTiming));
  }
  if (e != hipSuccess) {
    dd_set_error("dd_solver_create: %s", hipGetErrorString(e));
    dd_solver_destroy(s);
    return e == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP;
  }
  s->ddesc = dd;
  s->blk2prob = db2p;
  P.desc = dd;
  P.blk2prob = db2p;
  P.ctl = s->dctl;
  P.fused = s->fused ? 1 : 0;
  P.tiles = s->dtiles;
  e = precond_init(s);
  if (e != hipSuccess) {
    dd_set_error("dd_solver_create: %s", hipGetErrorString(e));
    dd_solver_destroy(s);
    return DD_EHIP;
  }
  *out = s;
  return DD_OK;
}

extern "C" size_t dd_solver_device_bytes(const dd_solver* s) { return s ? s->bytes : 0; }

extern "C" int dd_solver_elems_per_thread(const dd_solver* s) { return s ? s->R : 0; }

extern "C" dd_status dd_solver_workspace_bytes(const fdfd_op* const* ops, int nb,
                                               const dd_solver_opts* opts, size_t* bytes) {
  if (!bytes) { dd_set_error("dd_solver_workspace_bytes: bytes is NULL"); return DD_EINVAL; }
  *bytes = 0;
  dd_solver* s = nullptr;
  dd_status rc = solver_plan(ops, nb, opts, &s);
  if (rc != DD_OK) return rc;
  Arena A;
  ProbDesc* dd = nullptr;
  int* db2p = nullptr;
  layout_workspace(s, A, dd, db2p);
  *bytes = A.off;
  delete s;
  return DD_OK;
}

extern "C" size_t gmres_workspace_bytes(const fdfd_op* op, int k, int restart, dd_prec inner) {
  dd_solver_opts o;
  dd_solver_opts_default(&o);
  o.kmax = k;
  o.restart = restart;
  o.inner = inner;
  size_t b = 0;
  const fdfd_op* ops[1] = {op};
  return dd_solver_workspace_bytes(ops, 1, &o, &b) == DD_OK ? b : 0;
}

extern "C" dd_status dd_solver_bind(dd_solver* s, const fdfd_op* const* ops) {
  if (!s || !ops) { dd_set_error("dd_solver_bind: NULL argument"); return DD_EINVAL; }
  for (int p = 0; p < s->nb; ++p) {
    if (!ops[p] || ops[p]->nx != s->hdesc[p].nx || ops[p]->ny != s->hdesc[p].ny) {
      dd_set_error("dd_solver_bind: operator %d missing or of a different grid size", p);
      return DD_EINVAL;
    }
  }
  for (int p = 0; p < s->nb; ++p) {
    s->ops[p] = ops[p];
    fill_desc_op(s->hdesc[p], ops[p]);
    s->hdesc[p].k = 0;
    s->ksetup[p] = 0;
  }
  s->has_subspace = false;
  s->cycle_valid = false;
  DD_HIP_CHECK(hipMemcpy(s->ddesc, s->hdesc.data(), sizeof(ProbDesc) * s->nb, hipMemcpyHostToDevice));
  DD_HIP_CHECK(precond_init(s));
  return DD_OK;
}

template <typename T>
static void launch_setup(dd_solver* s, hipStream_t st) {
  const int nb = s->nb, K = s->o.kmax;
  PlanDev& P = s->P;
  int maxD = 0;
  for (auto& d : s->hdesc) maxD = std::max(maxD, d.Dp);
  const int gx = std::min(64, (maxD + DD_BLOCK - 1) / DD_BLOCK);
  k_copy_pad<T><<<dim3(gx, K, nb), DD_BLOCK, 0, st>>>(P, s->dU);
  k_stencil_multi<T><<<dim3(gx, K, nb), DD_BLOCK, 0, st>>>(P);
  for (int pass = 0; pass < 2; ++pass) {
    k_gram<T><<<dim3(P.GB, nb), DD_BLOCK, 0, st>>>(P);
    k_chol<<<nb, DD_BLOCK, 0, st>>>(P, pass);
    k_combine_multi<T><<<dim3(gx, nb), DD_BLOCK, 0, st>>>(P);
  }
}

extern "C" dd_status dd_solver_set_subspace(dd_solver* s, const void* const* U, const int* k,
                                            hipStream_t stream) {
  if (!s) { dd_set_error("dd_solver_set_subspace: NULL solver"); return DD_EINVAL; }
  std::vector<const void*> hU(s->nb, nullptr);
  bool any = false;
  for (int p = 0; p < s->nb; ++p) {
    int kp = (U && k) ? k[p] : 0;
    if (kp < 0 || kp > s->o.kmax) {
      dd_set_error("dd_solver_set_subspace: k[%d] = %d outside 0..kmax = %d", p, kp, s->o.kmax);
      return DD_EINVAL;
    }
    if (kp > 0 && !U[p]) {
      dd_set_error("dd_solver_set_subspace: U[%d] is NULL with k = %d", p, kp);
      return DD_EINVAL;
    }
    s->hdesc[p].k = kp;
    s->ksetup[p] = kp;
    hU[p] = kp > 0 ? U[p] : nullptr;
    any = any || kp > 0;
  }
  DD_HIP_CHECK(hipMemcpyAsync(s->ddesc, s->hdesc.data(), sizeof(ProbDesc) * s->nb,
                              hipMemcpyHostToDevice, stream));
  DD_HIP_CHECK(hipMemcpyAsync(s->dU, hU.data(), sizeof(void*) * s->nb, hipMemcpyHostToDevice,
                              stream));
  DD_HIP_CHECK(hipMemsetAsync(s->P.bad, 0, sizeof(unsigned long long) * s->nb, stream));
  DD_HIP_CHECK(hipMemsetAsync(s->P.keep, 0, sizeof(unsigned long long) * s->nb, stream));
  if (any) {
    if (s->o.inner == DD_C64) launch_setup<float>(s, stream);
    else launch_setup<double>(s, stream);
    DD_HIP_CHECK(hipGetLastError());
  }
  // the host arrays above are pageable: finish the copies before they go away
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  s->has_subspace = any;
  s->cycle_valid = false;
  return DD_OK;
}

static void prof_mark(dd_solver* s, int kind, hipStream_t st) {
  if (!s->prof || s->pused + 2 > (int)s->pev.size()) return;
  (void)hipEventRecord(s->pev[s->pused], st);
  s->pkind[s->pused / 2] = kind;
}
static void prof_end(dd_solver* s, hipStream_t st) {
  if (!s->prof || s->pused + 2 > (int)s->pev.size()) return;
  (void)hipEventRecord(s->pev[s->pused + 1], st);
  s->pused += 2;
}
// Adds the elapsed times of the recorded pairs (the stream has been
// synchronised by the caller) and recycles the events.
static void prof_collect(dd_solver* s) {
  for (int i = 0; i + 1 < s->pused; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->pev[i], s->pev[i + 1]) == hipSuccess) {
      const int kd = s->pkind[i / 2];
      s->ks.ms[kd] += ms;
      s->ks.launches[kd] += 1;
    }
  }
  s->pused = 0;
}

// Workgroups per problem for the reduction of a sweep's dot products: up to
// 32 value slices (about 256 workgroups in all), one where the adaptive
// second-pass test needs every coefficient of the first pass at once.
static int post_slices(const dd_solver* s, bool first_pass) {
  if (first_pass && s->P.reorth_mode == 2) return 1;
  return std::max(1, std::min(32, 256 / std::max(1, s->nb)));
}

// One Arnoldi step: matvec + first-pass dots, their reduction (which also
// decides the second pass), the optional second pass (only flagged problems
// do work in it), the final update + norm and the FP64 bookkeeping.
template <typename T, int R>
static void launch_step(dd_solver* s, int j, hipStream_t st) {
  const int g = s->nchunks, nb = s->nb;
  // a launch of few chunks (one problem) leaves most CUs idle: split its dot
  // products over up to four workgroups per chunk (groups of 16 vectors)
  const int ngrp = (s->o.kmax + j + 1 + 15) / 16;
  const dim3 gm(g, (g < s->ncu) ? std::min(4, ngrp) : 1);
  prof_mark(s, 0, st);
  if (s->o.precond != DD_PRECOND_NONE) k_matvec_dot<T, R, true><<<gm, DD_BLOCK, 0, st>>>(s->P, j);
  else k_matvec_dot<T, R, false><<<gm, DD_BLOCK, 0, st>>>(s->P, j);
  prof_end(s, st);
  k_post_dots<T><<<dim3(nb, post_slices(s, true)), DD_BLOCK, 0, st>>>(s->P, j, MODE_ARNOLDI, 0);
  if (s->P.reorth_mode != 0) {
    prof_mark(s, 1, st);
    k_update_dot<T, R><<<g, DD_BLOCK, 0, st>>>(s->P, j, MODE_ARNOLDI);
    prof_end(s, st);
    k_post_dots<T><<<dim3(nb, post_slices(s, false)), DD_BLOCK, 0, st>>>(s->P, j, MODE_ARNOLDI, 1);
  }
  prof_mark(s, 2, st);
  k_update_norm<T, R><<<g, DD_BLOCK, 0, st>>>(s->P, j, MODE_ARNOLDI, 0);
  prof_end(s, st);
  k_post_norm<T><<<nb, DD_BLOCK, 0, st>>>(s->P, j, MODE_ARNOLDI, 0);
}

// One fused Arnoldi step: the sweep (update of step j, matvec and dots of
// step j + 1) and its FP64 bookkeeping.
template <typename T>
static void launch_fused_step(dd_solver* s, int j, hipStream_t st) {
  const int nt = (int)s->htiles.size();
  const bool pc = s->o.precond != DD_PRECOND_NONE;
  prof_mark(s, 3, st);
  if (pc) k_fused_sweep<T, true><<<nt, DD_FUSED_THREADS, 0, st>>>(s->P, j);
  else k_fused_sweep<T, false><<<nt, DD_FUSED_THREADS, 0, st>>>(s->P, j);
  prof_end(s, st);
  k_post_fused<T><<<dim3(s->nb, post_slices(s, false)), DD_BLOCK, 0, st>>>(s->P, j, 0);
}

template <typename T, int R>
static void launch_any_step(dd_solver* s, int j, hipStream_t st) {
  if (s->fused) launch_fused_step<T>(s, j, st);
  else launch_step<T, R>(s, j, st);
}

// Projected start; it always takes the second pass unless one pass is
// requested, because a good subspace leaves r~ = r - C C^H r tiny against r.
template <typename T, int R>
static void launch_start(dd_solver* s, hipStream_t st) {
  const int g = s->nchunks, nb = s->nb;
  const int re = s->P.reorth_mode != 0;
  k_start_dot<T, R><<<g, DD_BLOCK, 0, st>>>(s->P);
  k_post_dots<T><<<nb, DD_BLOCK, 0, st>>>(s->P, 0, MODE_START, 0);
  if (re) {
    k_update_dot<T, R><<<g, DD_BLOCK, 0, st>>>(s->P, 0, MODE_START);
    k_post_dots<T><<<nb, DD_BLOCK, 0, st>>>(s->P, 0, MODE_START, 1);
  }
  k_update_norm<T, R><<<g, DD_BLOCK, 0, st>>>(s->P, 0, MODE_START, re);
  k_post_norm<T><<<nb, DD_BLOCK, 0, st>>>(s->P, 0, MODE_START, re);
}

// Captures (once) and launches the graph of Arnoldi steps [grp*ce, jend).
template <typename T, int R>
static dd_status launch_group_graph(dd_solver* s, int grp, int jend, hipStream_t st) {
  const int ce = s->o.check_every;
  if ((int)s->execs.size() <= grp) {
    s->execs.resize(grp + 1, nullptr);
    s->graphs.resize(grp + 1, nullptr);
  }
  if (!s->execs[grp]) {
    if (!s->cap) DD_HIP_CHECK(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    DD_HIP_CHECK(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
    for (int j = grp * ce; j < jend; ++j) launch_any_step<T, R>(s, j, s->cap);
    hipGraph_t g = nullptr;
    DD_HIP_CHECK(hipStreamEndCapture(s->cap, &g));
    hipGraphExec_t ex = nullptr;
    DD_HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    s->graphs[grp] = g;
    s->execs[grp] = ex;
  }
  DD_HIP_CHECK(hipGraphLaunch(s->execs[grp], st));
  return DD_OK;
}

template <typename T, int R>
static dd_status run_cycles(dd_solver* s, hipStream_t st) {
  const int nb = s->nb, m = s->o.restart, g = s->nchunks;
  const size_t stbytes = sizeof(int) * nb * ST_NI;
  int* snap[2] = {s->pinned, s->pinned + nb * ST_NI};
  bool first = true;
  for (;;) {
    k_residual<R><<<g, DD_BLOCK, 0, st>>>(s->P);
    k_post_residual<<<nb, DD_BLOCK, 0, st>>>(s->P, first ? 1 : 0);
    first = false;
    DD_HIP_CHECK(hipGetLastError());
    DD_HIP_CHECK(hipMemcpyAsync(snap[0], s->P.stI, stbytes, hipMemcpyDeviceToHost, st));
    DD_HIP_CHECK(hipStreamSynchronize(st));
    prof_collect(s);
    int active = 0;
    for (int p = 0; p < nb; ++p) active += snap[0][p * ST_NI + ST_ACTIVE];
    if (active == 0) break;
    launch_start<T, R>(s, st);
    if (s->fused) {
      // z_0 = A q~_0 (unscaled) and its dots; then the coefficients of step 0
      const int ngrp = (s->o.kmax + 1 + 15) / 16;
      const dim3 gm(s->nchunks, (s->nchunks < s->ncu) ? std::min(4, ngrp) : 1);
      prof_mark(s, 0, st);
      if (s->o.precond != DD_PRECOND_NONE) k_matvec_dot<T, R, true><<<gm, DD_BLOCK, 0, st>>>(s->P, 0);
      else k_matvec_dot<T, R, false><<<gm, DD_BLOCK, 0, st>>>(s->P, 0);
      prof_end(s, st);
      k_post_fused<T><<<dim3(nb, post_slices(s, false)), DD_BLOCK, 0, st>>>(s->P, 0, 1);
    }
    int pending = -1, grp = 0;
    const int ce = s->o.check_every;
    const bool graph = s->o.use_graph && !s->prof;
    for (int j = 0; j < m; ++j) {
      if (graph) {
        // one graph per group of ce steps; j is the group's first step
        if (j % ce == 0) {
          dd_status rc = launch_group_graph<T, R>(s, j / ce, std::min(m, j + ce), st);
          if (rc != DD_OK) return rc;
        }
        if ((j + 1) % ce != 0 && j + 1 < m) continue;
      } else {
        launch_any_step<T, R>(s, j, st);
      }
      if ((j + 1) % ce == 0 && j + 1 < m) {
        const int slot = (grp++) & 1;
        DD_HIP_CHECK(hipMemcpyAsync(snap[slot], s->P.stI, stbytes, hipMemcpyDeviceToHost, st));
        DD_HIP_CHECK(hipEventRecord(s->ev[slot], st));
        if (pending >= 0) {
          DD_HIP_CHECK(hipEventSynchronize(s->ev[pending]));
          int act = 0;
          for (int p = 0; p < nb; ++p) act += snap[pending][p * ST_NI + ST_ACTIVE];
          if (act == 0) break;
        }
        pending = slot;
      }
    }
    k_combine<T, R><<<g, DD_BLOCK, 0, st>>>(s->P);
    DD_HIP_CHECK(hipGetLastError());
  }
  return DD_OK;
}

template <typename T>
static dd_status run_cycles_T(dd_solver* s, hipStream_t st) {
  switch (s->R) {
    case 1: return run_cycles<T, 1>(s, st);
    case 2: return run_cycles<T, 2>(s, st);
    case 4: return run_cycles<T, 4>(s, st);
    default: return run_cycles<T, 8>(s, st);
  }
}

extern "C" dd_status dd_solver_solve(dd_solver* s, const void* const* b, const void* const* x0,
                                     double tol, int maxit, void* const* x, dd_info* info,
                                     hipStream_t stream) {
  if (!s || !b || !x) { dd_set_error("dd_solver_solve: NULL argument"); return DD_EINVAL; }
  if (!(tol >= 0.0) || maxit < 0) {
    dd_set_error("dd_solver_solve: need tol >= 0 and maxit >= 0");
    return DD_EINVAL;
  }
  const int nb = s->nb;
  for (int p = 0; p < nb; ++p) {
    if (!b[p] || !x[p]) { dd_set_error("dd_solver_solve: b[%d] or x[%d] is NULL", p, p); return DD_EINVAL; }
    s->hdesc[p].b = (const double2*)b[p];
    s->hdesc[p].x = (double2*)x[p];
  }
  DD_HIP_CHECK(hipMemcpyAsync(s->ddesc, s->hdesc.data(), sizeof(ProbDesc) * nb,
                              hipMemcpyHostToDevice, stream));
  for (int p = 0; p < nb; ++p) {
    const size_t bytes = sizeof(double2) * s->hdesc[p].D;
    const void* x0p = x0 ? x0[p] : nullptr;
    if (x0p) {
      if (x0p != x[p]) DD_HIP_CHECK(hipMemcpyAsync(x[p], x0p, bytes, hipMemcpyDeviceToDevice, stream));
    } else {
      DD_HIP_CHECK(hipMemsetAsync(x[p], 0, bytes, stream));
    }
  }
  {
    const double ctl[2] = {tol, (double)maxit};
    std::memcpy(s->hctl, ctl, sizeof(ctl));
    DD_HIP_CHECK(hipMemcpyAsync(s->dctl, s->hctl, sizeof(ctl), hipMemcpyHostToDevice, stream));
  }
  k_init_state<<<(nb + 255) / 256, 256, 0, stream>>>(s->P);
  DD_HIP_CHECK(hipGetLastError());
  s->cycle_valid = false;
  dd_status rc = (s->o.inner == DD_C64) ? run_cycles_T<float>(s, stream) : run_cycles_T<double>(s, stream);
  if (rc != DD_OK) return rc;
  s->cycle_valid = true;
  int* fin = s->pinned + 2 * nb * ST_NI;
  DD_HIP_CHECK(hipMemcpyAsync(fin, s->P.stI, sizeof(int) * nb * ST_NI, hipMemcpyDeviceToHost, stream));
  DD_HIP_CHECK(hipMemcpyAsync(s->pinnedD, s->P.stD, sizeof(double) * nb * SD_ND, hipMemcpyDeviceToHost, stream));
  DD_HIP_CHECK(hipMemcpyAsync(s->pinnedK, s->P.keep, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, stream));
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  dd_status out = DD_OK;
  if (s->prof) {
    // algorithmic bytes of the timed sweeps (inner precision ib bytes per
    // complex, eps eb bytes per cell): matvec + dots (2 ib + eb) D + ib D n;
    // second pass ib D (2n + 2); final update ib D (n + 2)
    const double ib = (double)inner_bytes(s->o.inner), eb = (s->o.inner == DD_C64) ? 4.0 : 8.0;
    for (int p = 0; p < nb; ++p) {
      const int* st = fin + p * ST_NI;
      const double* sd = s->pinnedD + p * SD_ND;
      const double D = s->hdesc[p].D, steps = st[ST_ITERS], st2 = st[ST_NREORTH];
      if (s->fused) {
        // first matvec of each cycle: (2 ib + eb) D + ib D (k + 1); fused
        // sweep of a step with n basis vectors: ib D (n + 3) + eb D
        const double cyc = st[ST_CYCLES], kk = s->hdesc[p].k;
        s->ks.bytes[0] += ((2 * ib + eb) + ib * (kk + 1)) * D * cyc;
        s->ks.bytes[3] += ib * D * (sd[SD_NSUM] + 3 * steps) + eb * D * steps;
      } else {
        s->ks.bytes[0] += (2 * ib + eb) * D * steps + ib * D * sd[SD_NSUM];
        s->ks.bytes[1] += ib * D * (2 * sd[SD_NSUM2] + 2 * st2);
        s->ks.bytes[2] += ib * D * (sd[SD_NSUM] + 2 * steps);
      }
    }
  }
  for (int p = 0; p < nb; ++p) {
    const int* st = fin + p * ST_NI;
    const double* sd = s->pinnedD + p * SD_ND;
    if (st[ST_FLAGS] & FLAG_ZERO_B)
      DD_HIP_CHECK(hipMemsetAsync(x[p], 0, sizeof(double2) * s->hdesc[p].D, stream));
    int kused = 0;
    if (s->has_subspace && s->ksetup[p] > 0) kused = __builtin_popcountll(s->pinnedK[p]);
    if (info) {
      dd_info& I = info[p];
      I.status = (st[ST_DONE] == DONE_CONVERGED) ? DD_OK : DD_NOT_CONVERGED;
      I.iters = st[ST_ITERS];
      I.restarts = st[ST_CYCLES];
      I.k_used = kused;
      I.fallback_plain = (s->ksetup[p] > 0 && kused == 0) ? 1 : 0;
      I.reorth_steps = st[ST_NREORTH];
      I.matvecs = (s->has_subspace ? s->ksetup[p] : 0) + st[ST_ITERS] + st[ST_CYCLES] + 1;
      I.rel_res_true = sd[SD_TRUE];
      I.rel_res_est = sd[SD_EST];
    }
    if (st[ST_DONE] == DONE_NONFINITE) {
      if (out == DD_OK || out == DD_NOT_CONVERGED) out = DD_ENONFINITE;
    } else if (st[ST_DONE] != DONE_CONVERGED && out == DD_OK) {
      out = DD_NOT_CONVERGED;
    }
  }
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  if (out == DD_ENONFINITE) dd_set_error("dd_solver_solve: non-finite right-hand side or residual");
  else if (out == DD_NOT_CONVERGED) dd_set_error("dd_solver_solve: iteration budget spent");
  return out;
}

// Tile-shape autotuner: times a few Arnoldi steps of each candidate
// elements-per-thread value on the given operators (right-hand sides of
// ones, restart and precision from opts) and returns the fastest.
extern "C" dd_status dd_solver_autotune(const fdfd_op* const* ops, int nb, const dd_solver_opts* opts,
                                        int* best, double* ms_per_step) {
  if (!ops || nb < 1 || !best) { dd_set_error("dd_solver_autotune: bad argument"); return DD_EINVAL; }
  dd_solver_opts o;
  dd_solver_opts_default(&o);
  if (opts) o = *opts;
  o.hist_cap = 0;
  o.kmax = 0;
  o.workspace = nullptr;      // candidates differ in size: each allocates its own
  o.workspace_bytes = 0;
  const int cands[4] = {1, 2, 4, 8};
  std::vector<double2*> bufs;
  std::vector<void*> bp(nb), xp(nb);
  dd_status rc = DD_OK;
  for (int p = 0; p < nb && rc == DD_OK; ++p) {
    double2 *b = nullptr, *x = nullptr;
    if (hipMalloc((void**)&b, sizeof(double2) * ops[p]->D) != hipSuccess ||
        hipMalloc((void**)&x, sizeof(double2) * ops[p]->D) != hipSuccess) {
      dd_set_error("dd_solver_autotune: hipMalloc failed");
      rc = DD_ENOMEM;
    }
    bufs.push_back(b);
    bufs.push_back(x);
    if (rc == DD_OK) k_fill_const<<<(ops[p]->D + 255) / 256, 256>>>(b, ops[p]->D, 1.0);
    bp[p] = b;
    xp[p] = x;
  }
  double bestms = 1e300;
  // one full cycle, so that the basis grows to its full length
  const int steps = o.restart;
  for (int ci = 0; ci < 4 && rc == DD_OK; ++ci) {
    o.elems_per_thread = cands[ci];
    dd_solver* s = nullptr;
    rc = dd_solver_create(ops, nb, &o, &s);
    if (rc != DD_OK) break;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    // warm-up (also captures the graphs), then a timed solve of `steps` steps
    dd_status r1 = dd_solver_solve(s, (const void* const*)bp.data(), nullptr, 0.0, steps, xp.data(), nullptr, 0);
    (void)hipEventRecord(e0, 0);
    dd_status r2 = dd_solver_solve(s, (const void* const*)bp.data(), nullptr, 0.0, steps, xp.data(), nullptr, 0);
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dd_solver_destroy(s);
    if (r1 < 0 || r2 < 0) { rc = r1 < 0 ? r1 : r2; break; }
    const double per = ms / steps;
    if (ms_per_step) ms_per_step[ci] = per;
    if (per < bestms) { bestms = per; *best = cands[ci]; }
  }
  for (double2* b : bufs)
    if (b) (void)hipFree(b);
  return rc;
}

extern "C" dd_status dd_solver_profile(dd_solver* s, int enable) {
  if (!s) { dd_set_error("dd_solver_profile: NULL solver"); return DD_EINVAL; }
  if (enable && s->pev.empty()) {
    const int n = 6 * s->o.restart + 8;
    s->pev.resize(n, nullptr);
    s->pkind.resize(n / 2 + 1, 0);
    for (auto& e : s->pev) DD_HIP_CHECK(hipEventCreate(&e));
  }
  s->prof = enable != 0;
  s->pused = 0;
  std::memset(&s->ks, 0, sizeof(s->ks));
  return DD_OK;
}

extern "C" dd_status dd_solver_kernel_stats(const dd_solver* s, dd_kernel_stats* out) {
  if (!s || !out) { dd_set_error("dd_solver_kernel_stats: NULL argument"); return DD_EINVAL; }
  *out = s->ks;
  return DD_OK;
}

extern "C" dd_status dd_solver_history(const dd_solver* s, int p, double* out, int cap, int* n) {
  if (!s || p < 0 || p >= s->nb || (!out && cap > 0)) {
    dd_set_error("dd_solver_history: bad argument");
    return DD_EINVAL;
  }
  int it = 0;
  DD_HIP_CHECK(hipMemcpy(&it, s->P.stI + p * ST_NI + ST_ITERS, sizeof(int), hipMemcpyDeviceToHost));
  const int cnt = std::min(std::min(it, s->o.hist_cap), cap);
  if (cnt > 0)
    DD_HIP_CHECK(hipMemcpy(out, s->P.hist + (size_t)p * s->o.hist_cap, sizeof(double) * cnt,
                           hipMemcpyDeviceToHost));
  if (n) *n = cnt;
  return DD_OK;
}

extern "C" dd_status dd_solver_debug_copy(const dd_solver* s, int p, int what, void* host_out,
                                          size_t bytes) {
  if (!s || p < 0 || p >= s->nb || !host_out) {
    dd_set_error("dd_solver_debug_copy: bad argument");
    return DD_EINVAL;
  }
  DD_HIP_CHECK(hipDeviceSynchronize());
  const ProbDesc& d = s->hdesc[p];
  const size_t ib = inner_bytes(s->o.inner);
  const int K = s->o.kmax, m = s->o.restart, k = d.k;
  char* dst = (char*)host_out;
  if (what == 0 || what == 1) {
    const int nvec = (what == 0) ? k : m + 1;
    const int slot0 = (what == 0) ? K - k : K;
    if (bytes != (size_t)nvec * d.D * ib) { dd_set_error("dd_solver_debug_copy: size mismatch"); return DD_EINVAL; }
    for (int v = 0; v < nvec; ++v)
      DD_HIP_CHECK(hipMemcpy(dst + (size_t)v * d.D * ib,
                             (const char*)d.basis + (size_t)(slot0 + v) * d.Dp * ib, d.D * ib,
                             hipMemcpyDeviceToHost));
    return DD_OK;
  }
  if (what == 2) {
    if (bytes != sizeof(double2) * m * (m + 1)) { dd_set_error("dd_solver_debug_copy: size mismatch"); return DD_EINVAL; }
    DD_HIP_CHECK(hipMemcpy(dst, s->P.Hraw + (size_t)p * m * (m + 1), bytes, hipMemcpyDeviceToHost));
    return DD_OK;
  }
  if (what == 3) {
    if (bytes != sizeof(double2) * m * k) { dd_set_error("dd_solver_debug_copy: size mismatch"); return DD_EINVAL; }
    for (int j = 0; j < m; ++j)
      DD_HIP_CHECK(hipMemcpy(dst + sizeof(double2) * j * k, s->P.Bc + ((size_t)p * m + j) * K,
                             sizeof(double2) * k, hipMemcpyDeviceToHost));
    return DD_OK;
  }
  if (what == 4) {
    if (bytes != sizeof(double2) * k * k) { dd_set_error("dd_solver_debug_copy: size mismatch"); return DD_EINVAL; }
    for (int a = 0; a < k; ++a)
      DD_HIP_CHECK(hipMemcpy(dst + sizeof(double2) * a * k, s->P.Rinv + ((size_t)p * K + a) * K,
                             sizeof(double2) * k, hipMemcpyDeviceToHost));
    return DD_OK;
  }
  dd_set_error("dd_solver_debug_copy: unknown array %d", what);
  return DD_EINVAL;
}

extern "C" dd_status gmres_solve_batched(const fdfd_op* const* ops, int nb, const void* const* b,
                                         const void* const* x0, const void* const* U, const int* k,
                                         double tol, int restart, int maxit,
                                         const dd_solver_opts* opts, void* const* x, dd_info* info,
                                         hipStream_t stream) {
  dd_solver_opts o;
  dd_solver_opts_default(&o);
  if (opts) o = *opts;
  o.restart = restart;
  int kmax = 0;
  if (U && k)
    for (int p = 0; p < nb; ++p) kmax = std::max(kmax, k[p]);
  o.kmax = std::max(o.kmax, kmax);
  dd_solver* s = nullptr;
  dd_status rc = dd_solver_create(ops, nb, &o, &s);
  if (rc != DD_OK) return rc;
  if (kmax > 0) {
    rc = dd_solver_set_subspace(s, U, k, stream);
    if (rc != DD_OK) { dd_solver_destroy(s); return rc; }
  }
  rc = dd_solver_solve(s, b, x0, tol, maxit, x, info, stream);
  dd_solver_destroy(s);
  return rc;
}

extern "C" dd_status gmres_solve(const fdfd_op* op, const void* b, const void* x0, const void* U,
                                 int k, double tol, int restart, int maxit,
                                 const dd_solver_opts* opts, void* x, dd_info* info,
                                 hipStream_t stream) {
  const fdfd_op* ops[1] = {op};
  const void* bs[1] = {b};
  const void* x0s[1] = {x0};
  const void* Us[1] = {U};
  int ks[1] = {U ? k : 0};
  void* xs[1] = {x};
  return gmres_solve_batched(ops, 1, bs, x0 ? x0s : nullptr, U ? Us : nullptr, U ? ks : nullptr, tol,
                             restart, maxit, opts, xs, info, stream);
}
