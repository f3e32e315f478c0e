// Host orchestration and C ABI of libpw (see include/pw.h).
//
// Owns the patch registry, device buffers, ghost and tile lists, the cover-flag
// arrays and the captured step graph; every step of the method runs in the HIP
// kernels of pw_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pw.h"
#include "pw_internal.h"
#include "pw_kernels.h"

using namespace pw;

// Staging memory of pw_get_state_noalloc: a file-scope device array, one copy
// per GPU (each device holds its own at its own address until the process
// ends).  Host code never uses the name `scratch` as an address: the address
// is resolved once per device with hipGetSymbolAddress (in pw_create, with the
// device current) and kept in g_scratch_ptr.
#define PW_NOALLOC_MAX_ELEMS (4u << 20)  // 4 Mi doubles = 32 MiB
static __device__ __align__(256) double scratch[PW_NOALLOC_MAX_ELEMS];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {nullptr};

struct pw_context {
  pw_config cfg;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // validation switch (environment variable PW_L2G_DIRECT=1 when the context is
  // created): every local->global point takes the direct gather from global
  // memory instead of the staged donor box; the values are the same bitwise
  bool l2g_direct = false;
  std::string err;
  std::vector<pw_patch_desc> desc;
  std::vector<PatchDev> hp;
  std::vector<void *> allocs;
  PatchDev *dP = nullptr;
  PoseDev *dPose = nullptr;  // 4 slots x np
  ExactDev hex[PW_MAXSV];
  ExactDev *dEx = nullptr;
  double *dVs = nullptr;
  int *dPts = nullptr;
  double *dT = nullptr;       // current time t_n
  double *dTx = nullptr;      // explicit time for eager calls
  unsigned long long *dCounters = nullptr;  // skip_local, skip_eff, skip_uncover, n_uncover, steps
  int *dErr = nullptr;
  // flags of the global patch
  long long gcells = 0;
  uint8_t *flag_cur = nullptr, *flag_new = nullptr, *t1 = nullptr, *t2 = nullptr, *live = nullptr;
  uint8_t *dbl = nullptr;  // cells claimed by two local patches (k_cover)
  int32_t *cover_cur = nullptr, *cover_new = nullptr;
  int2 *ulist = nullptr;  // cells that become live at the end of a step
  int *ucount = nullptr;
  // lists
  GhostRec *dLower = nullptr;
  int nLower = 0, nLowerGlobal = 0;
  // physical ghost cells of the global patch (outer ghosts that are not
  // periodic copies) and the lists of those covered by a local patch:
  // olist[0]/ocount[0] of the running step, olist[1]/ocount[1] of the next
  GhostRec *dPhys = nullptr;
  int nPhys = 0;
  int2 *olist[2] = {nullptr, nullptr};
  int *ocount[2] = {nullptr, nullptr};
  // Sommerfeld outer boundary: the global patch's outer ghost cells (evolved)
  GhostRec *dRad = nullptr;
  int nRad = 0;
  bool outer_ready = false;  // their values in u are set (state changes clear it)
  // analytic outer ghosts of the stage-0 buffer hold the exact solution at the
  // current time (each step's last stage writes them for the next step; state
  // changes clear it)
  bool outer0_ready = false;
  hipStream_t stream2 = nullptr;  // second branch of the overlapped step
  hipStream_t stream3 = nullptr;  // third branch: the next step's cover flags and lists
  hipEvent_t evFork = nullptr, evG[4] = {nullptr, nullptr, nullptr, nullptr},
             evL[4] = {nullptr, nullptr, nullptr, nullptr}, evE[4] = {nullptr, nullptr, nullptr, nullptr},
             evGL[4] = {nullptr, nullptr, nullptr, nullptr}, evS[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t evGhL = nullptr, evGhG = nullptr, evNext = nullptr;
  void *scratch_dev = nullptr;  // this device's copy of `scratch` (pw_get_state_noalloc)
  GBrick *dBricks = nullptr;
  int nBricks = 0;
  int32_t *efflist = nullptr, *effsorted = nullptr;
  int *effcount = nullptr;
  int nBuckets = 0;
  int *bkCnt = nullptr, *bkOff = nullptr, *bkRank = nullptr, *eBkt = nullptr, *eRank = nullptr;
  int2 *l2gItems = nullptr;  // local -> global work items (bucket runs), rebuilt with the flags
  int *l2gNItems = nullptr;
  FallbackRec *fbList[2] = {nullptr, nullptr};  // skipped points of the local / global part
  int *fbCount[2] = {nullptr, nullptr};
  long long fbCap = 0;
  uint8_t *dvalid[PW_NPTS] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // donor-valid bytes, P = 2 .. 6
  TileRec *dTiles = nullptr;
  int nTiles = 0;
  std::vector<int> tileOff, tileCnt;
  int nGlobalTiles = 0;
  int coordTiles[4] = {0, 0, 0, 0};  // local-patch tiles by topology: group t is [coordTiles[t], coordTiles[t+1])
  CoverJob *dJobs = nullptr;
  CoverBlk *dCoverBlk = nullptr;
  int nJobs = 0, nCoverBlk = 0;
  double *dStage = nullptr;  // staging for host copies
  long long stageCap = 0;
  double *dPartial = nullptr;
  bool layout_dirty = true, flags_valid = false;
  pw_tuning tune = {TUNE_TZ_GLOBAL, TUNE_TZ_LOCAL, TUNE_G2L_RUN, TUNE_L2G_RUN, PW_ORDER_BANDS, TUNE_CHAIN, TUNE_LOCAL_TILE, TUNE_GLOBAL_TILE};
  double t_host = 0.0;
  // first failure of a runtime call while a step is enqueued (event records and
  // waits between the step's streams); reported by pw_rk4_step
  hipError_t enq_err = hipSuccess;
  const char *enq_what = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  double graph_dt = 0.0;
  long long steps_done = 0;
  // per-kernel-class timing (eager path only)
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  struct Mark { int cls; hipEvent_t a, b; };
  std::vector<Mark> marks;
  double k_ms[PW_K_NCLASS] = {0};
  long long k_cnt[PW_K_NCLASS] = {0};
};

namespace {

pw_status fail(pw_context *c, pw_status code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, PW_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Record the first failing runtime call of an enqueue sequence.
void enq_check(pw_context *c, hipError_t e, const char *what) {
  if (e != hipSuccess && c->enq_err == hipSuccess) {
    c->enq_err = e;
    c->enq_what = what;
  }
}
#define ENQ(ctx, call) enq_check(ctx, (call), #call)

void *dalloc(pw_context *c, size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (c->cfg.dev_alloc) {
    p = c->cfg.dev_alloc((uint64_t)bytes, c->cfg.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->allocs.push_back(p);
  return p;
}

void dfree(pw_context *c, void *p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  if (c->cfg.dev_free) c->cfg.dev_free(p, c->cfg.alloc_user);
  else (void)hipFree(p);
}

void euler_zyz(const double e[3], double R[9]) {
  double ca = cos(e[0]), sa = sin(e[0]), cb = cos(e[1]), sb = sin(e[1]), cc = cos(e[2]), sc = sin(e[2]);
  // Rz(a) Ry(b) Rz(c)
  double A[3][3] = {{ca, -sa, 0}, {sa, ca, 0}, {0, 0, 1}};
  double B[3][3] = {{cb, 0, sb}, {0, 1, 0}, {-sb, 0, cb}};
  double C[3][3] = {{cc, -sc, 0}, {sc, cc, 0}, {0, 0, 1}};
  double T[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      T[i][j] = 0;
      for (int k = 0; k < 3; k++) T[i][j] += B[i][k] * C[k][j];
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0;
      for (int k = 0; k < 3; k++) s += A[i][k] * T[k][j];
      R[3 * i + j] = s;
    }
}

double bound_radius(const pw_patch_desc &d) {
  if (d.coord == PW_SPH) return d.hi[0];
  if (d.coord == PW_CYL) {
    const double zm = std::max(fabs(d.lo[2]), fabs(d.hi[2]));
    return sqrt(d.hi[0] * d.hi[0] + zm * zm);
  }
  double m = 0;
  for (int c = 0; c < 8; c++) {
    double y0 = (c & 1) ? d.hi[0] : d.lo[0], y1 = (c & 2) ? d.hi[1] : d.lo[1], y2 = (c & 4) ? d.hi[2] : d.lo[2];
    m = std::max(m, sqrt(y0 * y0 + y1 * y1 + y2 * y2));
  }
  return m;
}

uint32_t pack_ijk(int i, int j, int k) {
  return (uint32_t)(i + PW_NG) | ((uint32_t)(j + PW_NG) << 10) | ((uint32_t)(k + PW_NG) << 20);
}

bool mixed(const pw_context *c) { return c->cfg.precision == PW_MIXED || c->cfg.precision == PW_MIXED_INC; }
size_t stage_elem(const pw_context *c) { return mixed(c) ? sizeof(float) : sizeof(double); }
bool has_locals(const pw_context *c) { return c->hp.size() > 1; }
// The global patch's tile shape in effect, for the tile list and the launch
// alike: the two-rows-per-thread shape exists in the mixed modes only (and
// pw_set_tuning rejects it in FP64).
int global_tile_in_effect(const pw_context *c) {
  return (c->tune.global_tile == PW_TILE_128X8 && !mixed(c)) ? PW_TILE_128X4 : c->tune.global_tile;
}
// a buffer narrower than NG + 1 cells (the original Patchwork flags as an
// ablation): global->local stencils may reach effective ghosts
bool narrow_buffer(const pw_context *c) { return c->cfg.buffer_width < PW_NG + 1; }

hipEvent_t take_event(pw_context *c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Bracket the launches issued between begin/end with events when timing is on.
struct Timed {
  pw_context *c;
  int cls;
  hipEvent_t a = nullptr;
  Timed(pw_context *c_, int cls_) : c(c_), cls(cls_) {
    if (c->timing && cls >= 0) {
      a = take_event(c);
      (void)hipEventRecord(a, c->stream);
    }
  }
  ~Timed() {
    if (c->timing && cls >= 0) {
      hipEvent_t b = take_event(c);
      (void)hipEventRecord(b, c->stream);
      c->marks.push_back(pw_context::Mark{cls, a, b});
    }
  }
};

void harvest_marks(pw_context *c) {
  for (auto &m : c->marks) {
    float ms = 0;
    (void)hipEventSynchronize(m.b);
    (void)hipEventElapsedTime(&ms, m.a, m.b);
    c->k_ms[m.cls] += ms;
    c->k_cnt[m.cls] += 1;
    c->ev_free.push_back(m.a);
    c->ev_free.push_back(m.b);
  }
  c->marks.clear();
}

pw_status upload_layout(pw_context *c) {
  if (!c->layout_dirty) return PW_OK;
  if (c->hp.empty()) return fail(c, PW_ESTATE, "no global patch");
  int np = (int)c->hp.size();
  dfree(c, c->dP);
  dfree(c, c->dPose);
  c->dP = (PatchDev *)dalloc(c, sizeof(PatchDev) * np);
  c->dPose = (PoseDev *)dalloc(c, sizeof(PoseDev) * 4 * np);
  if (!c->dP || !c->dPose) return fail(c, PW_ENOMEM, "device allocation failed");
  HIPCHK(c, hipMemcpyAsync(c->dP, c->hp.data(), sizeof(PatchDev) * np, hipMemcpyHostToDevice, c->stream));

  // Lower-priority ghost cells (periodic copies, global outer ghosts) as a list;
  // the interpatch targets of every local patch as bricks of at most 8x8x3 cells
  // on its six faces (z faces span the full padded x-y range, y faces the full
  // padded x range, x faces the interior y-z range, so the faces are disjoint).
  std::vector<GhostRec> lower, rad, phys;
  std::vector<GBrick> bricks;
  const bool somm = c->cfg.outer_bc == PW_BC_SOMMERFELD;
  for (int pid = 0; pid < np; pid++) {
    const PatchDev &p = c->hp[pid];
    for (int k = -PW_NG; k < p.n[2] + PW_NG; k++)
      for (int j = -PW_NG; j < p.n[1] + PW_NG; j++)
        for (int i = -PW_NG; i < p.n[0] + PW_NG; i++) {
          int cc[3] = {i, j, k};
          bool inside = true, wrapped_inside = true;
          for (int a = 0; a < 3; a++) {
            inside = inside && cc[a] >= 0 && cc[a] < p.n[a];
            int w = p.periodic[a] ? ((cc[a] % p.n[a]) + p.n[a]) % p.n[a] : cc[a];
            wrapped_inside = wrapped_inside && w >= 0 && w < p.n[a];
          }
          if (inside) continue;
          if (p.is_global && !wrapped_inside && somm)
            rad.push_back(GhostRec{pid, pack_ijk(i, j, k)});
          else if (wrapped_inside || p.is_global)
            lower.push_back(GhostRec{pid, pack_ijk(i, j, k)});
          // covered physical ghosts (Sec. 2.4.2) are interpatch targets unless
          // the Sommerfeld variant evolves them
          if (p.is_global && !wrapped_inside && !somm && np > 1) phys.push_back(GhostRec{pid, pack_ijk(i, j, k)});
        }
    if (p.is_global) {
      c->nLowerGlobal = (int)lower.size();
      continue;
    }
    auto target = [&](int i, int j, int k) {
      int cc[3] = {i, j, k};
      bool inside = true, wrapped_inside = true;
      for (int a = 0; a < 3; a++) {
        inside = inside && cc[a] >= 0 && cc[a] < p.n[a];
        int w = p.periodic[a] ? ((cc[a] % p.n[a]) + p.n[a]) % p.n[a] : cc[a];
        wrapped_inside = wrapped_inside && w >= 0 && w < p.n[a];
      }
      return !inside && !wrapped_inside;
    };
    auto add = [&](int i0, int i1, int j0, int j1, int k0, int k1, int bi, int bj, int bk) {
      for (int k = k0; k < k1; k += bk)
        for (int j = j0; j < j1; j += bj)
          for (int i = i0; i < i1; i += bi) {
            GBrick b{pid, i, j, k, std::min(bi, i1 - i), std::min(bj, j1 - j), std::min(bk, k1 - k), 0};
            bool any = false;
            for (int z = b.k0; z < b.k0 + b.dk && !any; z++)
              for (int y = b.j0; y < b.j0 + b.dj && !any; y++)
                for (int x = b.i0; x < b.i0 + b.di && !any; x++) any = target(x, y, z);
            if (any) bricks.push_back(b);
          }
    };
    const int g = PW_NG;
    const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
    add(-g, n0 + g, -g, n1 + g, -g, 0, 8, 8, 3);        // z- face (with edges and corners)
    add(-g, n0 + g, -g, n1 + g, n2, n2 + g, 8, 8, 3);   // z+ face
    add(-g, n0 + g, -g, 0, 0, n2, 8, 3, 8);             // y- face
    add(-g, n0 + g, n1, n1 + g, 0, n2, 8, 3, 8);        // y+ face
    add(-g, 0, 0, n1, 0, n2, 3, 8, 8);                  // x- face
    add(n0, n0 + g, 0, n1, 0, n2, 3, 8, 8);             // x+ face
  }
  dfree(c, c->dRad);
  c->nRad = (int)rad.size();
  c->dRad = (GhostRec *)dalloc(c, sizeof(GhostRec) * std::max<size_t>(1, rad.size()));
  if (!c->dRad) return fail(c, PW_ENOMEM, "device allocation failed");
  if (!rad.empty()) HIPCHK(c, hipMemcpy(c->dRad, rad.data(), sizeof(GhostRec) * rad.size(), hipMemcpyHostToDevice));
  c->outer_ready = false;
  c->outer0_ready = false;
  dfree(c, c->dPhys);
  for (int m = 0; m < 2; m++) {
    dfree(c, c->olist[m]);
    dfree(c, c->ocount[m]);
  }
  c->nPhys = (int)phys.size();
  c->dPhys = (GhostRec *)dalloc(c, sizeof(GhostRec) * std::max<size_t>(1, phys.size()));
  for (int m = 0; m < 2; m++) {
    c->olist[m] = (int2 *)dalloc(c, sizeof(int2) * std::max<size_t>(1, phys.size()));
    c->ocount[m] = (int *)dalloc(c, sizeof(int));
    if (!c->olist[m] || !c->ocount[m]) return fail(c, PW_ENOMEM, "device allocation failed");
  }
  if (!c->dPhys) return fail(c, PW_ENOMEM, "device allocation failed");
  if (!phys.empty())
    HIPCHK(c, hipMemcpy(c->dPhys, phys.data(), sizeof(GhostRec) * phys.size(), hipMemcpyHostToDevice));
  launch_fill_i32(c->stream, c->ocount[0], 1, 0);
  launch_fill_i32(c->stream, c->ocount[1], 1, 0);
  dfree(c, c->dLower);
  dfree(c, c->dBricks);
  c->nLower = (int)lower.size();
  c->nBricks = (int)bricks.size();
  c->dLower = (GhostRec *)dalloc(c, sizeof(GhostRec) * std::max<size_t>(1, lower.size()));
  c->dBricks = (GBrick *)dalloc(c, sizeof(GBrick) * std::max<size_t>(1, bricks.size()));
  if (!c->dLower || !c->dBricks) return fail(c, PW_ENOMEM, "device allocation failed");
  if (!lower.empty())
    HIPCHK(c, hipMemcpy(c->dLower, lower.data(), sizeof(GhostRec) * lower.size(), hipMemcpyHostToDevice));
  if (!bricks.empty())
    HIPCHK(c, hipMemcpy(c->dBricks, bricks.data(), sizeof(GBrick) * bricks.size(), hipMemcpyHostToDevice));
  dfree(c, c->bkCnt);
  dfree(c, c->bkOff);
  dfree(c, c->bkRank);
  c->bkCnt = (int *)dalloc(c, sizeof(int) * std::max(1, c->nBuckets));
  c->bkOff = (int *)dalloc(c, sizeof(int) * std::max(1, c->nBuckets));
  c->bkRank = (int *)dalloc(c, sizeof(int) * std::max(1, c->nBuckets));
  if (!c->bkCnt || !c->bkOff || !c->bkRank) return fail(c, PW_ENOMEM, "device allocation failed");
  dfree(c, c->l2gItems);
  dfree(c, c->l2gNItems);
  // at most one partial item per bucket plus one per L2G_ITEM effective ghosts
  c->l2gItems = (int2 *)dalloc(c, sizeof(int2) * ((size_t)std::max(1, c->nBuckets) + (size_t)(c->gcells / L2G_ITEM) + 1));
  c->l2gNItems = (int *)dalloc(c, sizeof(int));
  if (!c->l2gItems || !c->l2gNItems) return fail(c, PW_ENOMEM, "device allocation failed");
  launch_fill_i32(c->stream, c->l2gNItems, 1, 0);
  {
    // bucket ids of each local patch follow a Morton curve through its
    // 8 x 8 x 4-cell buckets, so that consecutive buckets are spatial neighbours
    std::vector<int> rank(std::max(1, c->nBuckets), 0);
    for (int pid = 1; pid < np; pid++) {
      const PatchDev &p = c->hp[pid];
      const int nb = p.bkt_n[0] * p.bkt_n[1] * p.bkt_n[2];
      std::vector<std::pair<uint64_t, int>> key(nb);
      for (int b = 0; b < nb; b++) {
        const int bx = b % p.bkt_n[0], by = (b / p.bkt_n[0]) % p.bkt_n[1], bz = b / (p.bkt_n[0] * p.bkt_n[1]);
        uint64_t m = 0;
        for (int bit = 0; bit < 20; bit++)
          m |= ((uint64_t)((bx >> bit) & 1) << (3 * bit)) | ((uint64_t)((by >> bit) & 1) << (3 * bit + 1)) |
               ((uint64_t)((bz >> bit) & 1) << (3 * bit + 2));
        key[b] = {m, b};
      }
      std::sort(key.begin(), key.end());
      for (int r = 0; r < nb; r++) rank[p.bkt_base + key[r].second] = r;
    }
    HIPCHK(c, hipMemcpy(c->bkRank, rank.data(), sizeof(int) * rank.size(), hipMemcpyHostToDevice));
  }
  // fallback lists: every local ghost cell (local part) or every global cell (global part)
  long long nloc = 0;
  for (int pid = 1; pid < np; pid++) {
    const PatchDev &p = c->hp[pid];
    nloc += (long long)(p.n[0] + 2 * PW_NG) * (p.n[1] + 2 * PW_NG) * (p.n[2] + 2 * PW_NG);
  }
  long long cap = std::max(nloc, c->gcells);
  if (cap > c->fbCap) {
    for (int m = 0; m < 2; m++) {
      dfree(c, c->fbList[m]);
      dfree(c, c->fbCount[m]);
      c->fbList[m] = (FallbackRec *)dalloc(c, sizeof(FallbackRec) * cap);
      c->fbCount[m] = (int *)dalloc(c, sizeof(int));
      if (!c->fbList[m] || !c->fbCount[m]) return fail(c, PW_ENOMEM, "device allocation failed");
    }
    c->fbCap = cap;
  }

  // Tiles of every patch, grouped by patch and the patches by topology
  // (Cartesian, spherical, cylindrical; the global patch first).
  std::vector<TileRec> tiles;
  c->tileOff.assign(np, 0);
  c->tileCnt.assign(np, 0);
  // the global patch's tiles first, then those of the local patches grouped
  // by topology (Cartesian, spherical, cylindrical)
  auto add_tiles = [&](int pid) {
    const PatchDev &p = c->hp[pid];
    c->tileOff[pid] = (int)tiles.size();
    const bool sq = c->tune.local_tile == 1;
    const int gt = global_tile_in_effect(c);
    const int TX = pid == 0 ? (gt == 2 ? StageTile<true, 2>::TX : gt == 1 ? StageTile<true, 1>::TX : StageTile<true, 0>::TX)
                            : (sq ? StageTile<false, 1>::TX : StageTile<false, 0>::TX);
    const int TY = pid == 0 ? (gt == 2 ? StageTile<true, 2>::TY : gt == 1 ? StageTile<true, 1>::TY : StageTile<true, 0>::TY)
                            : (sq ? StageTile<false, 1>::TY : StageTile<false, 0>::TY);
    const int TZ = pid == 0 ? c->tune.tile_z_global : c->tune.tile_z_local;
    if (pid == 0 && c->tune.global_order == PW_ORDER_OCTANTS) {
      // the global patch in its eight octants (halves of the tile counts along
      // each axis), each z-chunk by z-chunk: the stage kernel hands each XCD a
      // contiguous eighth of the tiles, so every XCD works through one octant,
      // and only three faces of it are shared with another XCD's L2
      const int nx = (p.n[0] + TX - 1) / TX, ny = (p.n[1] + TY - 1) / TY, nzc = (p.n[2] + TZ - 1) / TZ;
      const int hx = (nx + 1) / 2, hy = (ny + 1) / 2, hz = (nzc + 1) / 2;
      for (int oz = 0; oz < 2; oz++)
        for (int oy = 0; oy < 2; oy++)
          for (int ox = 0; ox < 2; ox++)
            for (int zc = oz * hz; zc < std::min(nzc, (oz + 1) * hz); zc++)
              for (int yt = oy * hy; yt < std::min(ny, (oy + 1) * hy); yt++)
                for (int xt = ox * hx; xt < std::min(nx, (ox + 1) * hx); xt++)
                  tiles.push_back(TileRec{pid, xt * TX, yt * TY, zc * TZ, std::min(TZ, p.n[2] - zc * TZ)});
      c->tileCnt[pid] = (int)tiles.size() - c->tileOff[pid];
      return;
    }
    if (pid == 0) {
      // the global patch in eight bands of tile rows, each band z-chunk by
      // z-chunk: the stage kernel hands each XCD a contiguous run of tiles, so
      // every XCD works through one band of rows rather than one z-slab
      // (measured 6% faster per launch, with the same HBM fetch)
      const int ny = (p.n[1] + TY - 1) / TY, per = (ny + 7) / 8;
      for (int b0 = 0; b0 < ny; b0 += per)
        for (int z = 0; z < p.n[2]; z += TZ)
          for (int yt = b0; yt < std::min(ny, b0 + per); yt++)
            for (int x = 0; x < p.n[0]; x += TX) tiles.push_back(TileRec{pid, x, yt * TY, z, std::min(TZ, p.n[2] - z)});
      c->tileCnt[pid] = (int)tiles.size() - c->tileOff[pid];
      return;
    }
    for (int z = 0; z < p.n[2]; z += TZ)
      for (int y = 0; y < p.n[1]; y += TY)
        for (int x = 0; x < p.n[0]; x += TX) tiles.push_back(TileRec{pid, x, y, z, std::min(TZ, p.n[2] - z)});
    c->tileCnt[pid] = (int)tiles.size() - c->tileOff[pid];
  };
  add_tiles(0);
  c->nGlobalTiles = c->tileCnt[0];
  for (int t = 0; t < 3; t++) {
    c->coordTiles[t] = (int)tiles.size();
    for (int pid = 1; pid < np; pid++)
      if (c->hp[pid].coord == t) add_tiles(pid);
  }
  c->coordTiles[3] = (int)tiles.size();
  dfree(c, c->dTiles);
  c->nTiles = (int)tiles.size();
  c->dTiles = (TileRec *)dalloc(c, sizeof(TileRec) * tiles.size());
  if (!c->dTiles) return fail(c, PW_ENOMEM, "device allocation failed");
  HIPCHK(c, hipMemcpy(c->dTiles, tiles.data(), sizeof(TileRec) * tiles.size(), hipMemcpyHostToDevice));

  // Cover scans of the local patches.
  std::vector<CoverJob> jobs;
  const PatchDev &g = c->hp[0];
  std::vector<CoverBlk> cblk;
  for (int pid = 1; pid < np; pid++) {
    CoverJob J;
    J.patch = pid;
    J.radius = bound_radius(c->desc[pid]) * (1.0 + 1e-12) + 1e-12;
    long long tot = 1;
    for (int a = 0; a < 3; a++) {
      // a curvilinear global is scanned whole (its index box of a sphere is not simple)
      J.ext[a] = g.coord == CART ? (int)ceil(2.0 * J.radius * g.idx[a]) + 3 : g.n[a];
      tot *= J.ext[a];
    }
    if (tot >= (1LL << 31) - 256LL * COVER_CPT)
      return fail(c, PW_EINVAL, "the bounding box of a local patch spans 2^31 global cells or more");
    // workgroups of COVER_CPT x 256 consecutive box cells
    for (long long f = 0; f < tot; f += 256LL * COVER_CPT) cblk.push_back(CoverBlk{(int32_t)jobs.size(), (uint32_t)f});
    jobs.push_back(J);
  }
  dfree(c, c->dJobs);
  dfree(c, c->dCoverBlk);
  c->nJobs = (int)jobs.size();
  c->nCoverBlk = (int)cblk.size();
  c->dJobs = (CoverJob *)dalloc(c, sizeof(CoverJob) * std::max<size_t>(1, jobs.size()));
  c->dCoverBlk = (CoverBlk *)dalloc(c, sizeof(CoverBlk) * std::max<size_t>(1, cblk.size()));
  if (!c->dJobs || !c->dCoverBlk) return fail(c, PW_ENOMEM, "device allocation failed");
  if (!jobs.empty()) HIPCHK(c, hipMemcpy(c->dJobs, jobs.data(), sizeof(CoverJob) * jobs.size(), hipMemcpyHostToDevice));
  if (!cblk.empty())
    HIPCHK(c, hipMemcpy(c->dCoverBlk, cblk.data(), sizeof(CoverBlk) * cblk.size(), hipMemcpyHostToDevice));

  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
  }
  c->layout_dirty = false;
  c->flags_valid = false;
  return PW_OK;
}

pw_status set_time(pw_context *c, double *dptr, double t) {
  HIPCHK(c, hipMemcpyAsync(dptr, &t, sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PW_OK;
}

void enqueue_flags(pw_context *c, const PoseDev *pose_slot, hipStream_t st) {
  FlagsArgs a;
  a.P = c->dP;
  a.pose = pose_slot;
  a.jobs = c->dJobs;
  a.njobs = c->nJobs;
  a.blks = c->dCoverBlk;
  a.nblks = c->nCoverBlk;
  a.cover_new = c->cover_new;
  a.t1 = c->t1;
  a.t2 = c->t2;
  a.live = c->live;
  a.flag_new = c->flag_new;
  for (int d = 0; d < 3; d++) {
    a.n[d] = c->hp[0].n[d];
    a.wrap[d] = c->hp[0].periodic[d];
  }
  a.dbl = c->dbl;
  a.buffer = c->cfg.buffer_width;
  a.err = c->dErr;
  a.phys = c->dPhys;
  a.nphys = c->nPhys;
  a.olist = c->olist[1];
  a.ocount = c->ocount[1];
  launch_flags(st, a);
}

// Lists derived from the flags just computed (flag_new, cover_new): effective
// ghosts in donor-bucket order and donor validity.  They replace the lists of
// the running step, so they are enqueued after its last ghost fill and before
// the flags are made current by the finalize kernel.
void enqueue_post_flags(pw_context *c, const PoseDev *pose_slot, hipStream_t st) {
  PostFlagsArgs a;
  a.flag = c->flag_new;
  a.efflist = c->efflist;
  a.effcount = c->effcount;
  for (int m = 0; m < PW_NPTS; m++) {
    a.dvalid[m] = c->dvalid[m];
    a.Pvals[m] = 2 + m;
  }
  a.donor_effghost = narrow_buffer(c);
  a.t1 = c->t1;
  a.t2 = c->t2;
  for (int d = 0; d < 3; d++) {
    a.n[d] = c->hp[0].n[d];
    a.wrap[d] = c->hp[0].periodic[d];
  }
  launch_post_flags(st, a);
  L2GOrderArgs o;
  o.P = c->dP;
  o.pose = pose_slot;
  o.list = c->efflist;
  o.count = c->effcount;
  o.cover = c->cover_new;
  o.nbuckets = c->nBuckets;
  o.cnt = c->bkCnt;
  o.rank = c->bkRank;
  o.off = c->bkOff;
  o.ebkt = c->eBkt;
  o.erank = c->eRank;
  o.sorted = c->effsorted;
  o.out = c->efflist;  // the unordered list is not needed once scattered
  o.items = c->l2gItems;
  o.nitems = c->l2gNItems;
  launch_l2g_order(st, o);
}

void enqueue_finalize(pw_context *c, const PoseDev *pose_slot, int mode) {
  FinalizeArgs a;
  a.P = c->dP;
  a.pose = pose_slot;
  a.flag_cur = c->flag_cur;
  a.flag_new = c->flag_new;
  a.cover_cur = c->cover_cur;
  a.cover_new = c->cover_new;
  a.nsv = c->cfg.n_state_vectors;
  a.Pts = c->dPts;
  a.ex = c->dEx;
  a.vs = c->dVs;
  a.tdev = c->dT;
  a.mode = mode;
  a.counters = c->dCounters;
  for (int d = 0; d < 3; d++) a.n[d] = c->hp[0].n[d];
  a.ulist = c->ulist;
  a.ucount = c->ucount;
  a.olist_new = c->olist[1];
  a.ocount_new = c->ocount[1];
  a.olist_cur = c->olist[0];
  a.ocount_cur = c->ocount[0];
  a.nphys = c->nPhys;
  launch_finalize(c->stream, a);
}

bool analytic_outer_sv(const pw_context *c, int sv) {
  const PatchDev &g0 = c->hp[0];
  return g0.coord == CART && !g0.periodic[0] && !g0.periodic[1] && !g0.periodic[2] &&
         c->hex[sv].kind != PW_EXACT_NONE;
}

// Ghost fill of the buffers of `stage` (0: u) at time tdev[0] + tmul*dt.
void enqueue_ghosts(pw_context *c, int stage, const PoseDev *pose_slot, const double *tdev, double tmul, double dt,
                    int parts = GH_GLOBAL | GH_LOCAL, hipStream_t st = nullptr, bool fill_u = false,
                    int phases = PH_ALL, int sv_only = -1) {
  if (!st) st = c->stream;
  for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) {
    if (sv_only >= 0 && sv != sv_only) continue;
    GhostArgs a;
    a.P = c->dP;
    a.pose = pose_slot;
    a.parts = parts;
    a.phases = phases;
    // the outer ghosts of a Cartesian, non-periodic global patch with an exact
    // solution are analytic: the two midpoint stages (same time) share them, and
    // the last stage (time t_{n+1}) also writes those of the next step's first
    const bool analytic_outer = analytic_outer_sv(c, sv) && !fill_u;
    a.lower_dup = analytic_outer && stage == 1 ? 2 : (analytic_outer && stage == 3 ? 0 : -1);
    a.lower_skip_global = analytic_outer && (stage == 2 || stage == 0) ? 1 : 0;
    a.lower = c->dLower;
    a.n_lower = c->nLower;
    a.n_lower_global = c->nLowerGlobal;
    a.bricks = c->dBricks;
    a.n_bricks = has_locals(c) ? c->nBricks : 0;
    a.dvalid = c->dvalid[c->cfg.interp_points[sv] - 2];
    a.efflist = c->efflist;
    a.effcount = c->effcount;
    a.l2g_items = c->l2gItems;
    a.l2g_nitems = c->l2gNItems;
    a.cover = c->cover_cur;
    a.has_locals = has_locals(c);
    for (int d = 0; d < 3; d++) a.gn[d] = c->hp[0].n[d];
    a.sv = sv;
    a.stage = stage;
    a.stage_fp64 = !mixed(c) || fill_u;
    a.mixed = mixed(c);
    a.Pts = c->cfg.interp_points[sv];
    a.ex = c->dEx;
    a.v = c->cfg.wave_speed[sv];
    a.tdev = tdev;
    a.tmul = tmul;
    a.dt = dt;
    a.skips = c->dCounters;
    const int which = (parts & GH_LOCAL) ? 0 : 1;  // separate lists for concurrently running parts
    a.fb = c->fbList[which];
    a.fb_count = c->fbCount[which];
    a.g2l_run = c->tune.g2l_run;
    a.l2g_run = c->tune.l2g_run;
    a.l2g_first = narrow_buffer(c);
    a.global_curv = c->hp[0].coord != CART;
    a.g2l_exact_only = !(c->hp[0].sv_mask & (1u << sv)) && c->hex[sv].kind != PW_EXACT_NONE;
    a.l2g_direct = c->l2g_direct ? 1 : 0;
    a.gflag = c->flag_cur;
    a.phys = c->dPhys;
    a.olist = c->nPhys > 0 ? c->olist[0] : nullptr;
    a.nphys = c->nPhys;
    a.ocount = c->ocount[0];
    launch_ghosts(st, a);
  }
}

// One stage launch per topology over the tiles of all local patches of that
// topology.
void launch_local_groups(pw_context *c, StageArgs a, hipStream_t st, int topo_mask = 7) {
  for (int t = 0; t < 3; t++) {
    if (!((topo_mask >> t) & 1)) continue;
    a.tiles = c->dTiles + c->coordTiles[t];
    a.ntiles = c->coordTiles[t + 1] - c->coordTiles[t];
    a.coord = t;
    launch_stage(st, a);
  }
}

void enqueue_stage(pw_context *c, int stage, const PoseDev *pose_slot, double dt) {
  for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) {
    StageArgs a;
    a.P = c->dP;
    a.pose = pose_slot;
    a.gflag = has_locals(c) ? c->flag_cur : nullptr;
    a.sv = sv;
    a.stage = stage;
    a.mixed = mixed(c);
    a.inc = c->cfg.precision == PW_MIXED_INC;
    a.form = c->cfg.pi_form;
    a.local_tile = c->tune.local_tile;
    a.global_tile = global_tile_in_effect(c);
    a.dt = dt;
    a.v2 = c->cfg.wave_speed[sv] * c->cfg.wave_speed[sv];
    a.eps = c->cfg.ko_eps;
    bool all = true;
    for (auto &p : c->hp) all = all && (p.sv_mask & (1u << sv));
    if (c->cfg.schedule == PW_SCHED_PER_PATCH || !all) {
      for (size_t pid = 0; pid < c->hp.size(); pid++) {
        if (!(c->hp[pid].sv_mask & (1u << sv))) continue;
        a.tiles = c->dTiles + c->tileOff[pid];
        a.ntiles = c->tileCnt[pid];
        a.coord = c->hp[pid].coord;
        a.global = pid == 0;
        {
          Timed tg(c, pid == 0 ? PW_K_GSTAGE_S1 + stage : -1);
          launch_stage(c->stream, a);
        }
        if (pid == 0) launch_radiative(c->stream, c->dP, c->dRad, c->nRad, sv, stage, a.mixed, a.inc, dt, c->cfg.wave_speed[sv]);
      }
    } else {
      // batched: one launch over the global patch's tiles, then one over the
      // tiles of all local patches of each topology
      {
        Timed tg(c, PW_K_GSTAGE_S1 + stage);
        a.tiles = c->dTiles;
        a.ntiles = c->nGlobalTiles;
        a.coord = c->hp[0].coord;
        a.global = 1;
        launch_stage(c->stream, a);
      }
      launch_radiative(c->stream, c->dP, c->dRad, c->nRad, sv, stage, a.mixed, a.inc, dt, c->cfg.wave_speed[sv]);
      a.global = 0;
      launch_local_groups(c, a, c->stream);
    }
  }
}

// Stage kernels of the global patch (which = 1) or of the local patches (which =
// 2) of the topologies in topo_mask (bit 0 Cartesian, 1 spherical, 2 cylindrical).
void enqueue_stage_part(pw_context *c, int stage, const PoseDev *pose_slot, double dt, int which, hipStream_t st,
                        int topo_mask = 7) {
  for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) {
    StageArgs a;
    a.P = c->dP;
    a.pose = pose_slot;
    a.gflag = has_locals(c) ? c->flag_cur : nullptr;
    a.sv = sv;
    a.stage = stage;
    a.mixed = mixed(c);
    a.inc = c->cfg.precision == PW_MIXED_INC;
    a.form = c->cfg.pi_form;
    a.local_tile = c->tune.local_tile;
    a.global_tile = global_tile_in_effect(c);
    a.dt = dt;
    a.v2 = c->cfg.wave_speed[sv] * c->cfg.wave_speed[sv];
    a.eps = c->cfg.ko_eps;
    if (which == 1) {
      if (!(c->hp[0].sv_mask & (1u << sv))) continue;
      a.tiles = c->dTiles;
      a.ntiles = c->nGlobalTiles;
      a.coord = c->hp[0].coord;
      a.global = 1;
      launch_stage(st, a);
      launch_radiative(st, c->dP, c->dRad, c->nRad, sv, stage, a.mixed, a.inc, dt, c->cfg.wave_speed[sv]);
      continue;
    }
    a.global = 0;
    bool all = true;
    for (size_t pid = 1; pid < c->hp.size(); pid++) all = all && (c->hp[pid].sv_mask & (1u << sv));
    if (all) {
      launch_local_groups(c, a, st, topo_mask);
    } else {
      for (size_t pid = 1; pid < c->hp.size(); pid++) {
        if (!(c->hp[pid].sv_mask & (1u << sv)) || !((topo_mask >> c->hp[pid].coord) & 1)) continue;
        a.tiles = c->dTiles + c->tileOff[pid];
        a.ntiles = c->tileCnt[pid];
        a.coord = c->hp[pid].coord;
        launch_stage(st, a);
      }
    }
  }
}

// One step as two interleaved chains on two streams plus one for the flags.
//   X, the local chain: global -> local interpolation of stage s (it reads the
//     global stage s-1 output), its skipped points, the stage kernels of the
//     Cartesian local patches.
//   Y, the global chain: periodic copies of the local patches, local -> global
//     interpolation of stage s (it reads the local stage s-1 output), outer
//     ghosts, the global stage kernel.
//   The stage kernels of the curvilinear local patches (which need the global
//   -> local fill of X) go at the end of Y or before or after the Cartesian
//   ones on X (tuning parameter `chain`): which of them keeps the two chains
//   best overlapped depends on the mix of patches.
//   Z: the cover flags of the next step (they depend on the poses at t_{n+1}
//     only) while the stages run, and their lists once the last ghost fill of
//     this step is done.
// The uncover fill and the swap of the flags follow the last stage.  A buffer
// written at stage s was last read at stage s-2, by kernels that precede the
// writer through the global stage s-1 or the local stages s-1.
void enqueue_step_overlap(pw_context *c, double dt) {
  int np = (int)c->hp.size();
  hipStream_t X = c->stream, Y = c->stream2, Z = c->stream3;
  launch_pose(X, c->dP, np, c->dT, dt, c->dPose);
  ENQ(c, hipEventRecord(c->evFork, X));
  ENQ(c, hipStreamWaitEvent(Y, c->evFork, 0));
  ENQ(c, hipStreamWaitEvent(Z, c->evFork, 0));
  enqueue_flags(c, c->dPose + 2 * np, Z);
  static const int slot_of_stage[4] = {0, 1, 1, 2};
  static const double tmul[4] = {0.0, 0.5, 0.5, 1.0};
  const bool narrow = narrow_buffer(c);
  for (int s = 0; s < 4; s++) {
    const PoseDev *ps = c->dPose + slot_of_stage[s] * np;
    if (narrow) {
      // the global chain's local->global fill of this stage goes first; the
      // local chain's global->local stencils read the effective ghosts it wrote
      if (s > 0) ENQ(c, hipStreamWaitEvent(Y, c->evL[s - 1], 0));
      enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_GLOBAL, Y);
      if (s == 3) ENQ(c, hipEventRecord(c->evGhG, Y));
      ENQ(c, hipEventRecord(c->evE[s], Y));
      if (s > 0) ENQ(c, hipStreamWaitEvent(X, c->evG[s - 1], 0));
      ENQ(c, hipStreamWaitEvent(X, c->evE[s], 0));
      enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_LOCAL, X);
      if (s == 3) ENQ(c, hipEventRecord(c->evGhL, X));
      enqueue_stage_part(c, s, ps, dt, 2, X);
      ENQ(c, hipEventRecord(c->evL[s], X));
      enqueue_stage_part(c, s, ps, dt, 1, Y);
      ENQ(c, hipEventRecord(c->evG[s], Y));
      continue;
    }
    // X: global -> local interpolation (it reads the global stage s-1 output)
    // and its skipped points (they may copy interior cells of the curvilinear
    // local patches, written by their stage s-1 kernels on Y)
    // (state vector by state vector: they share the list of skipped points).
    // The periodic copies of stage 0 read the previous step's output only: they
    // go first on X, before the interpolation fills the GPU
    if (s == 0) enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_LOCAL, X, false, PH_LOWER);
    if (s > 0) ENQ(c, hipStreamWaitEvent(X, c->evG[s - 1], 0));
    for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) {
      enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_LOCAL, X, false, PH_INTERP, sv);
      if (sv == 0 && s > 0) ENQ(c, hipStreamWaitEvent(X, c->evS[s - 1], 0));
      enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_LOCAL, X, false, PH_FALLBACK, sv);
    }
    ENQ(c, hipEventRecord(c->evGL[s], X));
    if (s == 3) ENQ(c, hipEventRecord(c->evGhL, X));
    // Y: the periodic copies of the local patches (they read the local stage
    // s-1 output)
    if (s > 0) {
      ENQ(c, hipStreamWaitEvent(Y, c->evL[s - 1], 0));
      enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_LOCAL, Y, false, PH_LOWER);
      ENQ(c, hipEventRecord(c->evE[s], Y));
      ENQ(c, hipStreamWaitEvent(X, c->evE[s], 0));
    }
    // X: stage kernels of the Cartesian local patches, and of the curvilinear
    // ones before or after them unless they go on Y
    const int chain = c->tune.chain;
    if (chain == PW_CHAIN_LOCAL_BEFORE) enqueue_stage_part(c, s, ps, dt, 2, X, 6);
    enqueue_stage_part(c, s, ps, dt, 2, X, 1);
    if (chain == PW_CHAIN_LOCAL_AFTER) enqueue_stage_part(c, s, ps, dt, 2, X, 6);
    ENQ(c, hipEventRecord(c->evL[s], X));
    if (chain != PW_CHAIN_GLOBAL) ENQ(c, hipEventRecord(c->evS[s], X));
    // Y: local -> global interpolation, outer ghosts, global stage, then (if
    // they go here) the stage kernels of the curvilinear local patches, which
    // wait for X's fill
    enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_GLOBAL, Y);
    if (s == 3) ENQ(c, hipEventRecord(c->evGhG, Y));
    enqueue_stage_part(c, s, ps, dt, 1, Y);
    ENQ(c, hipEventRecord(c->evG[s], Y));
    if (chain == PW_CHAIN_GLOBAL) {
      ENQ(c, hipStreamWaitEvent(Y, c->evGL[s], 0));
      enqueue_stage_part(c, s, ps, dt, 2, Y, 6);
      ENQ(c, hipEventRecord(c->evS[s], Y));
    }
  }
  ENQ(c, hipStreamWaitEvent(Z, c->evGhL, 0));
  ENQ(c, hipStreamWaitEvent(Z, c->evGhG, 0));
  enqueue_post_flags(c, c->dPose + 2 * np, Z);
  ENQ(c, hipEventRecord(c->evNext, Z));
  ENQ(c, hipStreamWaitEvent(X, c->evG[3], 0));
  if (!narrow) ENQ(c, hipStreamWaitEvent(X, c->evS[3], 0));
  ENQ(c, hipStreamWaitEvent(X, c->evNext, 0));
  launch_advance_time(X, c->dT, dt, (long long *)c->dCounters);
  enqueue_finalize(c, c->dPose + 2 * np, 1);
}

void enqueue_step(pw_context *c, double dt) {
  int np = (int)c->hp.size();
  if (has_locals(c) && c->cfg.schedule == PW_SCHED_BATCHED && !c->timing && c->stream2 && c->stream3) {
    enqueue_step_overlap(c, dt);
    return;
  }
  {
    Timed tm(c, PW_K_POSE);
    launch_pose(c->stream, c->dP, np, c->dT, dt, c->dPose);
  }
  static const int slot_of_stage[4] = {0, 1, 1, 2};
  static const double tmul[4] = {0.0, 0.5, 0.5, 1.0};
  for (int s = 0; s < 4; s++) {
    const PoseDev *ps = c->dPose + slot_of_stage[s] * np;
    {
      Timed tm(c, PW_K_GHOST_S1 + s);
      if (c->timing && has_locals(c) && !narrow_buffer(c)) {
        // the interpatch kernels bracketed on their own (their skipped points and
        // the lower-priority fills follow each part, as in the overlapped step)
        for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) {
          {
            Timed tg(c, PW_K_G2L);
            enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_LOCAL, nullptr, false, PH_INTERP, sv);
          }
          enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_LOCAL, nullptr, false, PH_FALLBACK | PH_LOWER, sv);
          {
            Timed tl(c, PW_K_L2G);
            enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_GLOBAL, nullptr, false, PH_INTERP, sv);
          }
          enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt, GH_GLOBAL, nullptr, false, PH_FALLBACK | PH_LOWER, sv);
        }
      } else {
        enqueue_ghosts(c, s, ps, c->dT, tmul[s], dt);
      }
    }
    {
      Timed tm(c, PW_K_STAGE_S1 + s);
      enqueue_stage(c, s, ps, dt);
    }
  }
  launch_advance_time(c->stream, c->dT, dt, (long long *)c->dCounters);
  if (has_locals(c)) {
    {
      Timed tm(c, PW_K_FLAGS);
      enqueue_flags(c, c->dPose + 2 * np, c->stream);
      enqueue_post_flags(c, c->dPose + 2 * np, c->stream);
    }
    Timed tm(c, PW_K_FINALIZE);
    enqueue_finalize(c, c->dPose + 2 * np, 1);
  }
}

pw_status ensure_flags(pw_context *c) {
  pw_status rc = upload_layout(c);
  if (rc) return rc;
  if (c->flags_valid) return PW_OK;
  int np = (int)c->hp.size();
  if (has_locals(c)) {
    launch_pose(c->stream, c->dP, np, c->dT, 0.0, c->dPose);
    enqueue_flags(c, c->dPose, c->stream);
    enqueue_post_flags(c, c->dPose, c->stream);
    enqueue_finalize(c, c->dPose, 0);
    int err = 0;
    HIPCHK(c, hipMemcpyAsync(&err, c->dErr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (err) return fail(c, PW_EOVERLAP, "two local patches cover one global cell");
  }
  HIPCHK(c, hipGetLastError());
  c->flags_valid = true;
  return PW_OK;
}

pw_status check_error_flag(pw_context *c) {
  int err = 0;
  HIPCHK(c, hipMemcpyAsync(&err, c->dErr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (err) return fail(c, PW_EOVERLAP, "two local patches cover one global cell");
  return PW_OK;
}

// Device address of this device's `scratch` array: resolved once per device,
// with that device current.
pw_status resolve_scratch(pw_context *c) {
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(c, PW_EDEVICE, "device ordinal out of range for the staging table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(c, PW_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  c->scratch_dev = g_scratch_ptr[dev];
  return PW_OK;
}

pw_status ensure_stage(pw_context *c, long long n) {
  if (n <= c->stageCap) return PW_OK;
  dfree(c, c->dStage);
  c->dStage = (double *)dalloc(c, sizeof(double) * n);
  if (!c->dStage) return fail(c, PW_ENOMEM, "device allocation failed");
  c->stageCap = n;
  return PW_OK;
}

}  // namespace

extern "C" {

pw_status pw_create(const pw_config *cfg, pw_context **out) {
  if (!cfg || !out) return PW_EINVAL;
  *out = nullptr;
  if (cfg->n_state_vectors < 1 || cfg->n_state_vectors > PW_MAX_SV) return PW_EINVAL;
  if (cfg->precision != PW_FP64 && cfg->precision != PW_MIXED && cfg->precision != PW_MIXED_INC) return PW_EINVAL;
  if (cfg->buffer_width < 1 || cfg->buffer_width > 16) return PW_EINVAL;
  if (cfg->pi_form != PW_FORM_PAPER && cfg->pi_form != PW_FORM_FIRST_ORDER) return PW_EINVAL;
  if (cfg->outer_bc != PW_BC_EXACT && cfg->outer_bc != PW_BC_SOMMERFELD) return PW_EINVAL;
  for (int s = 0; s < cfg->n_state_vectors; s++) {
    if (cfg->interp_points[s] < 2 || cfg->interp_points[s] > 6) return PW_EINVAL;
    if (!(cfg->wave_speed[s] > 0)) return PW_EINVAL;
  }
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return PW_EINVAL;
  pw_context *c = new (std::nothrow) pw_context();
  if (!c) return PW_ENOMEM;
  c->cfg = *cfg;
  {
    const char *e = getenv("PW_L2G_DIRECT");
    c->l2g_direct = e && e[0] == '1' && e[1] == 0;
  }
  if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return PW_EDEVICE;
    }
    c->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->stream3, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->evFork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->evGhL, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->evGhG, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->evNext, hipEventDisableTiming) != hipSuccess) {
    pw_destroy(c);
    return PW_EDEVICE;
  }
  for (int s = 0; s < 4; s++)
    if (hipEventCreateWithFlags(&c->evG[s], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->evL[s], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->evE[s], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->evGL[s], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->evS[s], hipEventDisableTiming) != hipSuccess) {
      pw_destroy(c);
      return PW_EDEVICE;
    }
  for (int s = 0; s < PW_MAXSV; s++) memset(&c->hex[s], 0, sizeof(ExactDev));
  c->dEx = (ExactDev *)dalloc(c, sizeof(ExactDev) * PW_MAXSV);
  c->dVs = (double *)dalloc(c, sizeof(double) * PW_MAXSV);
  c->dPts = (int *)dalloc(c, sizeof(int) * PW_MAXSV);
  c->dT = (double *)dalloc(c, sizeof(double));
  c->dTx = (double *)dalloc(c, sizeof(double));
  c->dCounters = (unsigned long long *)dalloc(c, sizeof(unsigned long long) * 8);
  c->dErr = (int *)dalloc(c, sizeof(int));
  c->dPartial = (double *)dalloc(c, sizeof(double) * 1024 * DIAG_N);
  if (!c->dEx || !c->dVs || !c->dPts || !c->dT || !c->dTx || !c->dCounters || !c->dErr || !c->dPartial) {
    pw_destroy(c);
    return PW_ENOMEM;
  }
  double vs[PW_MAXSV] = {0, 0, 0, 0};
  int pts[PW_MAXSV] = {6, 6, 6, 6};
  for (int s = 0; s < cfg->n_state_vectors; s++) {
    vs[s] = cfg->wave_speed[s];
    pts[s] = cfg->interp_points[s];
  }
  unsigned long long zeros[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int zero = 0;
  double t0 = 0.0;
  if (hipMemcpy(c->dEx, c->hex, sizeof(ExactDev) * PW_MAXSV, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dVs, vs, sizeof(vs), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dPts, pts, sizeof(pts), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dT, &t0, sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dCounters, zeros, sizeof(zeros), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dErr, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    pw_destroy(c);
    return PW_EDEVICE;
  }
  if (resolve_scratch(c) != PW_OK) {
    pw_destroy(c);
    return PW_EDEVICE;
  }
  *out = c;
  return PW_OK;
}

pw_status pw_create_patch(pw_context *c, const pw_patch_desc *d, int32_t *id_out) {
  if (!c || !d) return PW_EINVAL;
  bool first = c->hp.empty();
  if ((d->is_global != 0) != first) return fail(c, PW_EINVAL, "the first patch, and only it, is the global patch");
  for (int a = 0; a < 3; a++) {
    if (d->n[a] < 1 || d->n[a] + 2 * PW_NG > 1023) return fail(c, PW_EINVAL, "cells per axis must be in [1, 1017]");
    if (!(d->hi[a] > d->lo[a])) return fail(c, PW_EINVAL, "empty numerical box");
    if (d->periodic[a] && d->n[a] < PW_NG) return fail(c, PW_EINVAL, "periodic axis needs at least 3 cells");
  }
  if (d->coord != PW_CART && d->coord != PW_SPH && d->coord != PW_CYL) return fail(c, PW_EINVAL, "unknown topology");
  if (d->motion < PW_STATIC || d->motion > PW_CIRCLE) return fail(c, PW_EINVAL, "unknown motion");
  if (d->motion == PW_CIRCLE && !(d->radius > 0)) return fail(c, PW_EINVAL, "circle motion needs radius > 0");
  if (first) {
    if ((d->coord != PW_CART && d->coord != PW_SPH) || d->motion != PW_STATIC || d->euler_zyz[0] != 0 ||
        d->euler_zyz[1] != 0 || d->euler_zyz[2] != 0 || d->c0[0] != 0 || d->c0[1] != 0 || d->c0[2] != 0 ||
        d->spin[0] != 0 || d->spin[1] != 0 || d->spin[2] != 0)
      return fail(c, PW_EINVAL, "the global patch is Cartesian or spherical, static, unrotated and at the origin");
    if (d->coord == PW_SPH && (d->periodic[0] || d->periodic[1]))
      return fail(c, PW_EINVAL, "a spherical global patch is periodic only along phi");
    if (c->cfg.outer_bc == PW_BC_SOMMERFELD &&
        (d->coord != PW_CART || d->periodic[0] || d->periodic[1] || d->periodic[2]))
      return fail(c, PW_EINVAL, "the Sommerfeld outer boundary needs a non-periodic Cartesian global patch");
  } else {
    const int phi_axis = d->coord == PW_SPH ? 2 : d->coord == PW_CYL ? 1 : -1;
    for (int a = 0; a < 3; a++)
      if (d->periodic[a] && a != phi_axis)
        return fail(c, PW_EINVAL, "local patches are periodic only along a spherical or cylindrical phi axis");
    if (d->coord != PW_CART && !(d->lo[0] > 0)) return fail(c, PW_EINVAL, "curvilinear patch needs r_min > 0");
    const PatchDev &g = c->hp[0];
    if (g.coord == CART && (g.periodic[0] || g.periodic[1] || g.periodic[2]))
      return fail(c, PW_EINVAL, "local patches need a non-periodic Cartesian global patch");
  }
  if (d->coord == PW_SPH) {
    double th_lo = d->lo[1] - PW_NG * (d->hi[1] - d->lo[1]) / d->n[1];
    double th_hi = d->hi[1] + PW_NG * (d->hi[1] - d->lo[1]) / d->n[1];
    double r_lo = d->lo[0] - PW_NG * (d->hi[0] - d->lo[0]) / d->n[0];
    if (!(th_lo > 0 && th_hi < M_PI && r_lo > 0)) return fail(c, PW_EINVAL, "spherical ghosts must avoid r=0 and the poles");
    if (d->periodic[2] && fabs(d->hi[2] - d->lo[2] - 2 * M_PI) > 1e-12)
      return fail(c, PW_EINVAL, "periodic phi axis must span 2 pi");
  }
  if (d->coord == PW_CYL) {
    double r_lo = d->lo[0] - PW_NG * (d->hi[0] - d->lo[0]) / d->n[0];
    if (!(r_lo > 0)) return fail(c, PW_EINVAL, "cylindrical ghosts must avoid the axis r=0");
    if (d->periodic[1] && fabs(d->hi[1] - d->lo[1] - 2 * M_PI) > 1e-12)
      return fail(c, PW_EINVAL, "periodic phi axis must span 2 pi");
  }
  unsigned mask_all = (1u << c->cfg.n_state_vectors) - 1u;
  if ((d->sv_mask & ~mask_all) || d->sv_mask == 0) return fail(c, PW_EINVAL, "bad state-vector mask");
  if (!first && c->hp.size() >= 4096) return fail(c, PW_EINVAL, "too many patches");

  PatchDev p;
  memset(&p, 0, sizeof(p));
  p.coord = d->coord;
  p.is_global = d->is_global ? 1 : 0;
  p.motion = d->motion;
  for (int a = 0; a < 3; a++) {
    p.n[a] = d->n[a];
    p.periodic[a] = d->periodic[a] ? 1 : 0;
    p.lo[a] = d->lo[a];
    p.hi[a] = d->hi[a];
    p.dx[a] = (d->hi[a] - d->lo[a]) / d->n[a];
    p.idx[a] = 1.0 / p.dx[a];
    p.c0[a] = d->c0[a];
    p.vel[a] = d->vel[a];
    p.spin[a] = d->spin[a];
  }
  p.radius = d->radius;
  p.omega = d->motion == PW_CIRCLE ? d->speed / d->radius : 0.0;
  p.phase = d->phase;
  euler_zyz(d->euler_zyz, p.R);
  p.sv_mask = d->sv_mask;
  p.bkt_base = 0;
  for (int a = 0; a < 3; a++) p.bkt_n[a] = first ? 0 : (a == 2 ? (p.n[a] + 3) / 4 : (p.n[a] + 7) / 8);
  if (!first) {
    const PatchDev &last = c->hp.back();
    p.bkt_base = last.bkt_base + last.bkt_n[0] * last.bkt_n[1] * last.bkt_n[2];
  }
  p.pitch = ((PW_OX + p.n[0] + PW_NG) + 31) / 32 * 32;
  p.rows = p.n[1] + 2 * PW_NG;
  p.slabs = p.n[2] + 2 * PW_NG;
  p.slab = (long long)p.pitch * p.rows;
  p.fstride = p.slab * p.slabs;
  long long nel = 5 * p.fstride;
  // the kernels address the five fields of a patch with 32-bit element offsets
  if (nel > (long long)UINT32_MAX)
    return fail(c, PW_EINVAL, "a patch's five padded fields must hold fewer than 2^32 elements (about 925^3 cells)");
  if (p.coord != CART) {
    const int nt = 2 * (p.n[1] + p.n[2] + 4 * PW_NG);
    double *tab = (double *)dalloc(c, sizeof(double) * nt);
    if (!tab) return fail(c, PW_ENOMEM, "device allocation failed");
    launch_trig_table(c->stream, p.n[1], p.n[2], p.lo[1], p.dx[1], p.lo[2], p.dx[2], tab);
    p.trig = tab;
  }
  for (int s = 0; s < c->cfg.n_state_vectors; s++) {
    if (!(d->sv_mask & (1u << s))) continue;
    p.u[s] = (double *)dalloc(c, sizeof(double) * nel);
    p.acc[s] = (double *)dalloc(c, sizeof(double) * nel);
    p.va[s] = dalloc(c, stage_elem(c) * nel);
    p.vb[s] = dalloc(c, stage_elem(c) * nel);
    if (!p.u[s] || !p.acc[s] || !p.va[s] || !p.vb[s]) return fail(c, PW_ENOMEM, "device allocation failed");
    launch_fill_f64(c->stream, p.u[s], nel, NAN);
    launch_fill_f64(c->stream, p.acc[s], nel, NAN);
    if (mixed(c)) {
      p.us[s] = (float *)dalloc(c, sizeof(float) * nel);
      if (!p.us[s]) return fail(c, PW_ENOMEM, "device allocation failed");
      launch_fill_f32(c->stream, p.us[s], nel, NAN);
      launch_fill_f32(c->stream, (float *)p.va[s], nel, NAN);
      launch_fill_f32(c->stream, (float *)p.vb[s], nel, NAN);
    } else {
      launch_fill_f64(c->stream, (double *)p.va[s], nel, NAN);
      launch_fill_f64(c->stream, (double *)p.vb[s], nel, NAN);
    }
  }
  if (first) {
    c->gcells = (long long)p.n[0] * p.n[1] * p.n[2];
    c->flag_cur = (uint8_t *)dalloc(c, c->gcells);
    c->flag_new = (uint8_t *)dalloc(c, c->gcells);
    c->dbl = (uint8_t *)dalloc(c, c->gcells);
    c->t1 = (uint8_t *)dalloc(c, c->gcells);
    c->t2 = (uint8_t *)dalloc(c, c->gcells);
    c->live = (uint8_t *)dalloc(c, c->gcells);
    c->cover_cur = (int32_t *)dalloc(c, sizeof(int32_t) * c->gcells);
    c->cover_new = (int32_t *)dalloc(c, sizeof(int32_t) * c->gcells);
    c->ulist = (int2 *)dalloc(c, sizeof(int2) * c->gcells);
    c->ucount = (int *)dalloc(c, sizeof(int));
    c->efflist = (int32_t *)dalloc(c, sizeof(int32_t) * c->gcells);
    c->effsorted = (int32_t *)dalloc(c, sizeof(int32_t) * c->gcells);
    c->eBkt = (int *)dalloc(c, sizeof(int) * c->gcells);
    c->eRank = (int *)dalloc(c, sizeof(int) * c->gcells);
    c->effcount = (int *)dalloc(c, sizeof(int));
    if (!c->effsorted || !c->eBkt || !c->eRank) return fail(c, PW_ENOMEM, "device allocation failed");
    for (int m = 0; m < PW_NPTS; m++) {
      bool used = false;
      for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) used = used || c->cfg.interp_points[sv] == 2 + m;
      c->dvalid[m] = used ? (uint8_t *)dalloc(c, c->gcells) : nullptr;
      if (used && !c->dvalid[m]) return fail(c, PW_ENOMEM, "device allocation failed");
    }
    if (!c->flag_cur || !c->flag_new || !c->dbl || !c->t1 || !c->t2 || !c->live || !c->cover_cur || !c->cover_new || !c->ulist || !c->ucount ||
        !c->efflist || !c->effcount)
      return fail(c, PW_ENOMEM, "device allocation failed");
    launch_fill_u8(c->stream, c->flag_cur, c->gcells, LIVE);
    launch_fill_u8(c->stream, c->flag_new, c->gcells, LIVE);
    launch_fill_i32(c->stream, c->cover_cur, c->gcells, -1);
    launch_fill_i32(c->stream, c->cover_new, c->gcells, -1);
  }
  HIPCHK(c, hipGetLastError());
  c->hp.push_back(p);
  c->desc.push_back(*d);
  c->nBuckets = p.bkt_base + p.bkt_n[0] * p.bkt_n[1] * p.bkt_n[2];
  c->layout_dirty = true;
  c->flags_valid = false;
  if (id_out) *id_out = (int32_t)c->hp.size() - 1;
  return PW_OK;
}

pw_status pw_set_exact(pw_context *c, int32_t sv, const pw_exact_desc *ex) {
  if (!c || !ex || sv < 0 || sv >= c->cfg.n_state_vectors) return PW_EINVAL;
  ExactDev e;
  memset(&e, 0, sizeof(e));
  e.kind = ex->kind;
  if (ex->kind == PW_EXACT_PLANE) {
    e.amp = ex->amp;
    e.offset = ex->offset;
    e.phase = ex->phase;
    for (int a = 0; a < 3; a++) e.kappa[a] = ex->kappa[a];
    e.knorm = sqrt(e.kappa[0] * e.kappa[0] + e.kappa[1] * e.kappa[1] + e.kappa[2] * e.kappa[2]);
  } else if (ex->kind == PW_EXACT_GAUSS) {
    if (ex->n_pulses < 0 || ex->n_pulses > PW_MAX_PULSES) return fail(c, PW_EINVAL, "too many pulses");
    e.n = ex->n_pulses;
    for (int g = 0; g < e.n; g++) {
      if (!(ex->pulse_width[g] > 0)) return fail(c, PW_EINVAL, "pulse width must be > 0");
      e.pa[g] = ex->pulse_amp[g];
      e.pw[g] = ex->pulse_width[g];
      for (int a = 0; a < 3; a++) e.px[g][a] = ex->pulse_center[g][a];
    }
  } else if (ex->kind != PW_EXACT_NONE) {
    return fail(c, PW_EINVAL, "unknown exact-solution kind");
  }
  c->hex[sv] = e;
  // whether the outer ghosts are analytic is part of the captured step: recapture
  c->layout_dirty = true;
  c->outer0_ready = false;
  HIPCHK(c, hipMemcpyAsync(c->dEx + sv, &c->hex[sv], sizeof(ExactDev), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PW_OK;
}

pw_status pw_init_exact(pw_context *c, double t0) {
  if (!c) return PW_EINVAL;
  pw_status rc = upload_layout(c);
  if (rc) return rc;
  rc = set_time(c, c->dT, t0);
  if (rc) return rc;
  int np = (int)c->hp.size();
  launch_pose_at(c->stream, c->dP, np, t0, c->dPose + 3 * np);
  for (int pid = 0; pid < np; pid++)
    for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) {
      if (!(c->hp[pid].sv_mask & (1u << sv)) || c->hex[sv].kind == PW_EXACT_NONE) continue;
      long long ncell = (long long)c->hp[pid].n[0] * c->hp[pid].n[1] * c->hp[pid].n[2];
      launch_init_exact(c->stream, c->dP, c->dPose + 3 * np, pid, sv, c->dEx, c->cfg.wave_speed[sv], t0, ncell);
    }
  HIPCHK(c, hipGetLastError());
  c->t_host = t0;
  c->flags_valid = false;
  c->outer_ready = false;
  c->outer0_ready = false;
  return PW_OK;
}

pw_status pw_set_state(pw_context *c, int32_t pid, int32_t sv, const double *src, int64_t n, int32_t is_dev,
                       double t0) {
  if (!c || !src || pid < 0 || pid >= (int)c->hp.size() || sv < 0 || sv >= c->cfg.n_state_vectors) return PW_EINVAL;
  const PatchDev &p = c->hp[pid];
  if (!(p.sv_mask & (1u << sv))) return fail(c, PW_EINVAL, "patch does not carry this state vector");
  long long need = 5LL * p.n[0] * p.n[1] * p.n[2];
  if (n != need) return fail(c, PW_EINVAL, "element count does not match 5*n0*n1*n2");
  pw_status rc = upload_layout(c);
  if (rc) return rc;
  const double *dsrc = src;
  if (!is_dev) {
    rc = ensure_stage(c, need);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->dStage, src, sizeof(double) * need, hipMemcpyHostToDevice, c->stream));
    dsrc = c->dStage;
  }
  launch_unpack(c->stream, c->dP, pid, sv, dsrc, need);
  HIPCHK(c, hipGetLastError());
  rc = set_time(c, c->dT, t0);
  if (rc) return rc;
  c->t_host = t0;
  c->flags_valid = false;
  c->outer_ready = false;
  c->outer0_ready = false;
  return PW_OK;
}

static pw_status get_common(pw_context *c, int32_t pid, int32_t sv, double *dst, int64_t n, int32_t is_dev, int full) {
  if (!c || !dst || pid < 0 || pid >= (int)c->hp.size() || sv < 0 || sv >= c->cfg.n_state_vectors) return PW_EINVAL;
  const PatchDev &p = c->hp[pid];
  if (!(p.sv_mask & (1u << sv))) return fail(c, PW_EINVAL, "patch does not carry this state vector");
  int g = full ? 2 * PW_NG : 0;
  long long need = 5LL * (p.n[0] + g) * (p.n[1] + g) * (p.n[2] + g);
  if (n != need) return fail(c, PW_EINVAL, "element count does not match");
  pw_status rc = upload_layout(c);
  if (rc) return rc;
  double *ddst = dst;
  if (!is_dev) {
    rc = ensure_stage(c, need);
    if (rc) return rc;
    ddst = c->dStage;
  }
  launch_pack(c->stream, c->dP, pid, sv, ddst, need, full);
  HIPCHK(c, hipGetLastError());
  if (!is_dev) HIPCHK(c, hipMemcpyAsync(dst, ddst, sizeof(double) * need, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PW_OK;
}

pw_status pw_get_state(pw_context *c, int32_t pid, int32_t sv, double *dst, int64_t n, int32_t is_dev) {
  return get_common(c, pid, sv, dst, n, is_dev, 0);
}

// pw_get_state into host memory without any allocation: the packed state goes
// through this device's static staging array.
pw_status pw_get_state_noalloc(pw_context *c, int32_t pid, int32_t sv, double *dst, int64_t n) {
  if (!c || !dst || pid < 0 || pid >= (int)c->hp.size() || sv < 0 || sv >= c->cfg.n_state_vectors) return PW_EINVAL;
  const PatchDev &p = c->hp[pid];
  if (!(p.sv_mask & (1u << sv))) return fail(c, PW_EINVAL, "patch does not carry this state vector");
  const long long need = 5LL * p.n[0] * p.n[1] * p.n[2];
  if (n != need) return fail(c, PW_EINVAL, "element count does not match 5*n0*n1*n2");
  if (need > (long long)PW_NOALLOC_MAX_ELEMS)
    return fail(c, PW_EINVAL, "the patch's state exceeds the static staging array of pw_get_state_noalloc (" +
                                  std::to_string(PW_NOALLOC_MAX_ELEMS) + " values); use pw_get_state");
  if (c->layout_dirty || !c->scratch_dev)
    return fail(c, PW_ESTATE, "the patch layout is not on the device yet (call pw_init_exact, pw_set_state, "
                              "pw_get_state or pw_rk4_step once first)");
  double *stage = (double *)c->scratch_dev;
  launch_pack(c->stream, c->dP, pid, sv, stage, need, 0);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(dst, stage, sizeof(double) * need, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PW_OK;
}

pw_status pw_get_state_full(pw_context *c, int32_t pid, int32_t sv, double *dst, int64_t n) {
  return get_common(c, pid, sv, dst, n, 0, 1);
}

pw_status pw_get_flags(pw_context *c, uint8_t *flags, int32_t *cover, int64_t n) {
  if (!c || !flags) return PW_EINVAL;
  if (c->hp.empty()) return fail(c, PW_ESTATE, "no global patch");
  if (n != c->gcells) return fail(c, PW_EINVAL, "cell count does not match the global patch");
  pw_status rc = ensure_flags(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(flags, c->flag_cur, c->gcells, hipMemcpyDeviceToHost, c->stream));
  if (cover)
    HIPCHK(c, hipMemcpyAsync(cover, c->cover_cur, sizeof(int32_t) * c->gcells, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PW_OK;
}

// Sommerfeld outer boundary: before the first step on a new state, the outer
// ghosts of u (and of its FP32 copy) take the lower-priority value at the
// current time; from then on they are evolved with the state.
pw_status ensure_outer(pw_context *c) {
  if (c->cfg.outer_bc != PW_BC_SOMMERFELD || c->outer_ready) return PW_OK;
  pw_status rc = upload_layout(c);
  if (rc) return rc;
  const int np = (int)c->hp.size();
  launch_pose_at(c->stream, c->dP, np, c->t_host, c->dPose + 3 * np);
  for (int sv = 0; sv < c->cfg.n_state_vectors; sv++) {
    launch_fill_list(c->stream, c->dP, c->dPose + 3 * np, c->dRad, c->nRad, sv, 1, c->dEx, c->cfg.wave_speed[sv],
                     c->dT);
    if (mixed(c))
      launch_fill_list(c->stream, c->dP, c->dPose + 3 * np, c->dRad, c->nRad, sv, 0, c->dEx,
                       c->cfg.wave_speed[sv], c->dT);
  }
  HIPCHK(c, hipGetLastError());
  c->outer_ready = true;
  return PW_OK;
}

// The analytic outer ghosts of the stage-0 buffer at the current time, unless
// the last step wrote them (the step itself does not: its first stage reads them).
pw_status ensure_outer0(pw_context *c) {
  if (c->outer0_ready) return PW_OK;
  const int np = (int)c->hp.size();
  launch_pose_at(c->stream, c->dP, np, c->t_host, c->dPose + 3 * np);
  for (int sv = 0; sv < c->cfg.n_state_vectors; sv++)
    if (analytic_outer_sv(c, sv) && (c->hp[0].sv_mask & (1u << sv)))
      launch_fill_list(c->stream, c->dP, c->dPose + 3 * np, c->dLower, c->nLowerGlobal, sv, mixed(c) ? 0 : 1, c->dEx,
                       c->cfg.wave_speed[sv], c->dT);
  HIPCHK(c, hipGetLastError());
  c->outer0_ready = true;
  return PW_OK;
}

pw_status pw_exchange_ghosts(pw_context *c, double t) {
  if (!c) return PW_EINVAL;
  c->outer0_ready = false;  // it writes u, not the FP32 copy, at a time of the caller's choosing
  pw_status rc = ensure_flags(c);
  if (rc) return rc;
  rc = ensure_outer(c);
  if (rc) return rc;
  int np = (int)c->hp.size();
  rc = set_time(c, c->dTx, t);
  if (rc) return rc;
  launch_pose_at(c->stream, c->dP, np, t, c->dPose + 3 * np);
  // fills the ghosts of u itself (FP64) in both precision modes
  enqueue_ghosts(c, 0, c->dPose + 3 * np, c->dTx, 0.0, 0.0, GH_GLOBAL | GH_LOCAL, nullptr, true);
  HIPCHK(c, hipGetLastError());
  return PW_OK;
}

pw_status pw_rk4_step(pw_context *c, double dt, int32_t nsteps) {
  if (!c || !(dt > 0) || nsteps < 0) return PW_EINVAL;
  if (c->hp.empty()) return fail(c, PW_ESTATE, "no global patch");
  // The NG+1 buffer lets a patch cross at most one global cell per step; a wider
  // buffer B relaxes that to B - NG cells (Sec. 2.4.2).  The narrower buffers of
  // the ablation keep the one-cell bound.
  const double cells_per_step = std::max(1, c->cfg.buffer_width - PW_NG);
  const PatchDev &g = c->hp[0];
  double hmin = std::min(g.dx[0], std::min(g.dx[1], g.dx[2]));
  if (g.coord == SPH)  // smallest physical cell edge of a spherical shell
    hmin = std::min(g.dx[0], g.lo[0] * std::min(g.dx[1], std::min(sin(g.lo[1]), sin(g.hi[1])) * g.dx[2]));
  for (size_t pid = 1; pid < c->hp.size(); pid++) {
    const pw_patch_desc &d = c->desc[pid];
    double sp = 0;
    if (d.motion == PW_LINEAR) sp = sqrt(d.vel[0] * d.vel[0] + d.vel[1] * d.vel[1] + d.vel[2] * d.vel[2]);
    if (d.motion == PW_CIRCLE) sp = fabs(d.speed);
    // a spinning patch: points at distance rho from the centre move at |spin| rho more
    sp += sqrt(d.spin[0] * d.spin[0] + d.spin[1] * d.spin[1] + d.spin[2] * d.spin[2]) * bound_radius(d);
    if (sp * dt >= cells_per_step * hmin)
      return fail(c, PW_EMOTION, "a patch moves buffer_width - NG global cells or more within a step");
  }
  pw_status rc = ensure_flags(c);
  if (rc) return rc;
  rc = ensure_outer(c);
  if (rc) return rc;
  rc = ensure_outer0(c);
  if (rc) return rc;
  bool graph = c->cfg.use_graph && c->cfg.schedule == PW_SCHED_BATCHED && !c->timing;
  if (graph && (c->gexec == nullptr || c->graph_dt != dt)) {
    if (c->gexec) {
      (void)hipGraphExecDestroy(c->gexec);
      (void)hipGraphDestroy(c->graph);
      c->gexec = nullptr;
    }
    c->enq_err = hipSuccess;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    enqueue_step(c, dt);
    // every fork joined and nothing invalidated the capture: its status is
    // still active here, and each event record and wait succeeded
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    unsigned long long cid = 0;
    const hipError_t qe = hipStreamGetCaptureInfo(c->stream, &cs, &cid);
    hipGraph_t captured = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->stream, &captured);
    if (c->enq_err != hipSuccess || qe != hipSuccess || cs != hipStreamCaptureStatusActive || ee != hipSuccess ||
        captured == nullptr) {
      if (captured) (void)hipGraphDestroy(captured);
      (void)hipGetLastError();
      std::string why = c->enq_err != hipSuccess ? std::string(c->enq_what) + ": " + hipGetErrorString(c->enq_err)
                        : qe != hipSuccess        ? std::string("hipStreamGetCaptureInfo: ") + hipGetErrorString(qe)
                        : cs != hipStreamCaptureStatusActive ? std::string("the step capture was invalidated")
                                                             : std::string("hipStreamEndCapture: ") + hipGetErrorString(ee);
      return fail(c, PW_EDEVICE, "capturing the step graph failed: " + why);
    }
    c->graph = captured;
    HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    c->graph_dt = dt;
  }
  for (int n = 0; n < nsteps; n++) {
    if (graph) {
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    } else {
      c->enq_err = hipSuccess;
      enqueue_step(c, dt);
      if (c->enq_err != hipSuccess)
        return fail(c, PW_EDEVICE, std::string(c->enq_what) + ": " + hipGetErrorString(c->enq_err));
    }
    c->t_host = c->t_host + dt;
  }
  HIPCHK(c, hipGetLastError());
  c->steps_done += nsteps;
  return PW_OK;
}

pw_status pw_get_tuning(pw_context *c, pw_tuning *out) {
  if (!c || !out) return PW_EINVAL;
  *out = c->tune;
  return PW_OK;
}

pw_status pw_set_tuning(pw_context *c, const pw_tuning *t) {
  if (!c || !t) return PW_EINVAL;
  if (t->global_order != PW_ORDER_BANDS && t->global_order != PW_ORDER_OCTANTS)
    return fail(c, PW_EINVAL, "tuning parameter out of range");
  if (t->chain < PW_CHAIN_GLOBAL || t->chain > PW_CHAIN_LOCAL_BEFORE)
    return fail(c, PW_EINVAL, "tuning parameter out of range");
  if (t->local_tile != PW_TILE_32X8 && t->local_tile != PW_TILE_16X16)
    return fail(c, PW_EINVAL, "tuning parameter out of range");
  if (t->global_tile != PW_TILE_32X8 && t->global_tile != PW_TILE_128X4 && t->global_tile != PW_TILE_128X8)
    return fail(c, PW_EINVAL, "tuning parameter out of range");
  if (t->global_tile == PW_TILE_128X8 && !mixed(c))
    return fail(c, PW_EINVAL, "global tile 128x8 (two rows per thread) exists in the mixed modes only");
  if (t->tile_z_global < 1 || t->tile_z_global > 512 || t->tile_z_local < 1 || t->tile_z_local > 512 ||
      t->g2l_run < 1 || t->g2l_run > 64 || t->l2g_run < 1 || t->l2g_run > 64)
    return fail(c, PW_EINVAL, "tuning parameter out of range");
  c->tune = *t;
  c->layout_dirty = true;  // tile lists are rebuilt and the step graph re-captured
  return PW_OK;
}

// Coordinate search over the tuning parameters, each candidate timed with HIP
// events over steps_per_trial steps (after one untimed step, which also captures
// the step graph): the tile depths and the global tile order on a grid, then the
// other global tile shape (with the global tile depths), the chain of the
// curvilinear local stages, the other local tile shape (with the local tile
// depths), the brick run and the group run.
pw_status pw_autotune(pw_context *c, double dt, int32_t steps_per_trial, pw_tuning *best) {
  if (!c || !(dt > 0) || steps_per_trial < 1) return PW_EINVAL;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, PW_EDEVICE, "event creation failed");
  }
  pw_status rc = PW_OK;
  auto trial = [&](const pw_tuning &t, float &ms) -> pw_status {
    pw_status r = pw_set_tuning(c, &t);
    if (r) return r;
    r = pw_rk4_step(c, dt, 1);
    if (r) return r;
    if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, PW_EDEVICE, "event record failed");
    r = pw_rk4_step(c, dt, steps_per_trial);
    if (r) return r;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return fail(c, PW_EDEVICE, "event timing failed");
    return check_error_flag(c);
  };
  pw_tuning cur = c->tune, bestT = cur;
  float bestMs = 3.0e38f, ms = 0.0f;
  static const int tzg[3] = {16, 32, 64}, tzl[3] = {4, 8, 16}, runs_g2l[3] = {4, 8, 16}, runs_l2g[3] = {2, 4, 8};
  const pw_tuning base0 = bestT;
  for (int o = 0; o < 2 && !rc; o++)
    for (int a = 0; a < 3 && !rc; a++)
      for (int b = 0; b < 3 && !rc; b++) {
        pw_tuning t = base0;
        t.global_order = o;
        t.tile_z_global = tzg[a];
        t.tile_z_local = tzl[b];
        rc = trial(t, ms);
        if (!rc && ms < bestMs) { bestMs = ms; bestT = t; }
      }
  // the other global tile shapes, with the global tile depths again
  const pw_tuning base0b = bestT;
  for (int sh = 0; sh < 3 && !rc; sh++) {
    if (sh == base0b.global_tile || (sh == PW_TILE_128X8 && !mixed(c))) continue;
    for (int a = 0; a < 3 && !rc; a++) {
      pw_tuning t = base0b;
      t.global_tile = sh;
      t.tile_z_global = tzg[a];
      rc = trial(t, ms);
      if (!rc && ms < bestMs) { bestMs = ms; bestT = t; }
    }
  }
  if (has_locals(c)) {
    const pw_tuning base1 = bestT;
    for (int a = 0; a < 3 && !rc; a++) {
      if (a == base1.chain) continue;
      pw_tuning t = base1;
      t.chain = a;
      rc = trial(t, ms);
      if (!rc && ms < bestMs) { bestMs = ms; bestT = t; }
    }
    // the other local tile shape, with the local tile depths again
    const pw_tuning base1b = bestT;
    for (int b = 0; b < 3 && !rc; b++) {
      pw_tuning t = base1b;
      t.local_tile = 1 - base1b.local_tile;
      t.tile_z_local = tzl[b];
      rc = trial(t, ms);
      if (!rc && ms < bestMs) { bestMs = ms; bestT = t; }
    }
    const pw_tuning base = bestT;
    for (int a = 0; a < 3 && !rc; a++) {
      pw_tuning t = base;
      t.g2l_run = runs_g2l[a];
      rc = trial(t, ms);
      if (!rc && ms < bestMs) { bestMs = ms; bestT = t; }
    }
    const pw_tuning base2 = bestT;
    for (int a = 0; a < 3 && !rc; a++) {
      pw_tuning t = base2;
      t.l2g_run = runs_l2g[a];
      rc = trial(t, ms);
      if (!rc && ms < bestMs) { bestMs = ms; bestT = t; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    (void)pw_set_tuning(c, &cur);
    return rc;
  }
  rc = pw_set_tuning(c, &bestT);
  if (!rc && best) *best = bestT;
  return rc;
}

pw_status pw_get_time(const pw_context *c, double *t) {
  if (!c || !t) return PW_EINVAL;
  *t = c->t_host;
  return PW_OK;
}

pw_status pw_diagnostics(pw_context *c, int32_t pid, int32_t sv, pw_diag *out) {
  if (!c || !out || pid < 0 || pid >= (int)c->hp.size() || sv < 0 || sv >= c->cfg.n_state_vectors) return PW_EINVAL;
  if (!(c->hp[pid].sv_mask & (1u << sv))) return fail(c, PW_EINVAL, "patch does not carry this state vector");
  pw_status rc = ensure_flags(c);
  if (rc) return rc;
  rc = check_error_flag(c);
  if (rc) return rc;
  int np = (int)c->hp.size();
  launch_pose_at(c->stream, c->dP, np, c->t_host, c->dPose + 3 * np);
  const int nb = 1024;
  launch_diag(c->stream, c->dP, c->dPose + 3 * np, pid, sv, has_locals(c) ? c->flag_cur : nullptr, c->dEx,
              c->cfg.wave_speed[sv], c->t_host, c->dPartial, nb);
  HIPCHK(c, hipGetLastError());
  std::vector<double> h((size_t)nb * DIAG_N);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->dPartial, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double acc[DIAG_N];
  for (int x = 0; x < DIAG_N; x++) acc[x] = 0;
  for (int b = 0; b < nb; b++)
    for (int x = 0; x < DIAG_N; x++) {
      double v = h[(size_t)b * DIAG_N + x];
      bool mx = (x < 5) || (x >= 10 && x < 15) || x >= 24;
      acc[x] = mx ? std::max(acc[x], v) : acc[x] + v;
    }
  for (int f = 0; f < 5; f++) {
    out->max_abs[f] = acc[f];
    out->sum_sq[f] = acc[5 + f];
    out->err_max[f] = acc[10 + f];
    out->err_sum_sq[f] = acc[15 + f];
  }
  out->int_rel_err = acc[20];
  out->live_cells = acc[21];
  out->volume = acc[22];
  out->energy = acc[23];
  for (int a = 0; a < 3; a++) out->constraint_max[a] = acc[24 + a];
  return PW_OK;
}

pw_status pw_counters(pw_context *c, pw_counters_t *out) {
  if (!c || !out) return PW_EINVAL;
  if (c->dCounters == nullptr) return fail(c, PW_ESTATE, "no counters");
  unsigned long long h[8];
  HIPCHK(c, hipMemcpyAsync(h, c->dCounters, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out->skip_local = (int64_t)h[0];
  out->skip_eff = (int64_t)h[1];
  out->skip_uncover = (int64_t)h[2];
  out->n_uncover = (int64_t)h[3];
  out->steps = (int64_t)h[4];
  out->skip_outer = (int64_t)h[5];
  out->n_outer = (int64_t)h[6];
  return check_error_flag(c);
}

pw_status pw_live_cells(pw_context *c, int64_t *out) {
  if (!c || !out) return PW_EINVAL;
  if (c->hp.empty()) return fail(c, PW_ESTATE, "no global patch");
  pw_status rc = ensure_flags(c);
  if (rc) return rc;
  std::vector<uint8_t> f(c->gcells);
  HIPCHK(c, hipMemcpyAsync(f.data(), c->flag_cur, c->gcells, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  long long glive = 0;
  for (long long x = 0; x < c->gcells; x++) glive += f[x] == LIVE;
  long long tot = 0;
  for (size_t pid = 0; pid < c->hp.size(); pid++) {
    const PatchDev &p = c->hp[pid];
    long long cells = pid == 0 ? glive : (long long)p.n[0] * p.n[1] * p.n[2];
    tot += cells * __builtin_popcount(p.sv_mask);
  }
  *out = tot;
  return PW_OK;
}

pw_status pw_enable_timing(pw_context *c, int32_t on) {
  if (!c) return PW_EINVAL;
  c->timing = on != 0;
  return PW_OK;
}

pw_status pw_kernel_times(pw_context *c, double *total_ms, int64_t *count) {
  if (!c || !total_ms || !count) return PW_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  harvest_marks(c);
  for (int k = 0; k < PW_K_NCLASS; k++) {
    total_ms[k] = c->k_ms[k];
    count[k] = c->k_cnt[k];
    c->k_ms[k] = 0;
    c->k_cnt[k] = 0;
  }
  return PW_OK;
}

const char *pw_last_error(const pw_context *c) { return c ? c->err.c_str() : "null context"; }

void pw_destroy(pw_context *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->stream2) (void)hipStreamSynchronize(c->stream2);
  if (c->stream3) (void)hipStreamSynchronize(c->stream3);
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    (void)hipGraphDestroy(c->graph);
  }
  harvest_marks(c);
  for (auto e : c->ev_free) (void)hipEventDestroy(e);
  std::vector<void *> all = c->allocs;
  for (void *p : all) dfree(c, p);
  if (c->stream2) {
    (void)hipStreamSynchronize(c->stream2);
    (void)hipStreamDestroy(c->stream2);
  }
  if (c->stream3) (void)hipStreamDestroy(c->stream3);
  if (c->evFork) (void)hipEventDestroy(c->evFork);
  if (c->evGhL) (void)hipEventDestroy(c->evGhL);
  if (c->evGhG) (void)hipEventDestroy(c->evGhG);
  if (c->evNext) (void)hipEventDestroy(c->evNext);
  for (int s = 0; s < 4; s++) {
    if (c->evG[s]) (void)hipEventDestroy(c->evG[s]);
    if (c->evL[s]) (void)hipEventDestroy(c->evL[s]);
    if (c->evE[s]) (void)hipEventDestroy(c->evE[s]);
    if (c->evGL[s]) (void)hipEventDestroy(c->evGL[s]);
    if (c->evS[s]) (void)hipEventDestroy(c->evS[s]);
  }
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
