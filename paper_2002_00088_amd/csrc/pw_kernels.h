// Launch interface between the host orchestration and the HIP kernels of libpw.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pw_internal.h"

// Stage-kernel tiles: TX x TY columns per workgroup; the number of planes a
// workgroup marches through (the tile depth) is a run-time tuning parameter,
// one for the global patch and one for local patches.
#ifndef STAGE_GTX
#define STAGE_GTX 32
#endif
#ifndef STAGE_GTY
#define STAGE_GTY 8
#endif
// Tile shapes, run-time tuning parameters.  Global patch: SH = 0 tiles of
// STAGE_GTX x STAGE_GTY columns (32 x 8), SH = 1 tiles of 128 x 4 on 512 threads
// (longer contiguous rows per load), SH = 2 tiles of 128 x 8 on 512 threads, each
// thread holding two rows of the tile (RY = 2: half the halo cells per cell of
// SH = 1, twice the loads in flight per thread).  Local patches: SH = 0 tiles of
// 32 x 8, SH = 1 tiles of 16 x 16 (narrower tiles waste fewer columns on patches
// of 24-96 cells and have a smaller halo per cell, 1.89 against 2.08).
template <bool GLOB, int SH = 0>
struct StageTile {
  static constexpr int TX = GLOB ? (SH >= 1 ? 128 : STAGE_GTX) : (SH == 1 ? 16 : 32);
  static constexpr int TY = GLOB ? (SH == 1 ? 4 : SH == 2 ? 8 : STAGE_GTY) : (SH == 1 ? 16 : 8);
  static constexpr int RY = (GLOB && SH == 2) ? 2 : 1;  // tile rows per thread
  static constexpr int PX = TX + 6, PY = TY + 6, PW = PX * PY;  // LDS plane with a 3-cell halo
  static constexpr int THREADS = TX * TY / RY;
  static_assert(TY % RY == 0, "whole rows per thread");
};
// Tuning defaults (measured on the batched 256^3 + 64-patch workload).
#define TUNE_TZ_GLOBAL 32
#define TUNE_TZ_LOCAL 8
#define TUNE_G2L_RUN 8
#define TUNE_L2G_RUN 4
#define TUNE_CHAIN 0
#define TUNE_LOCAL_TILE 0
#define TUNE_GLOBAL_TILE 1
#define DIAG_N 27
#define BRICK_THREADS 192
#ifndef BRICK_LDS_BYTES
#define BRICK_LDS_BYTES 30720
#endif
#ifndef L2G_BLOCKS
#define L2G_BLOCKS 4096  // workgroups of the local -> global kernel (a multiple of 8)
#endif
#define L2G_THREADS 192  // threads of a local -> global workgroup
#define L2G_ITEM 64      // entries of a local -> global work item (at most one donor bucket)
#ifndef L2G_LDS_BYTES
#define L2G_LDS_BYTES 39424  // donor box: 1971 cells of five FP32 values (a 14 x 14 x 10 box fits)
#endif
#define BUCKET_SORT_LDS 4096

namespace pw {

struct TileRec {
  int32_t patch, x0, y0, z0, nz;  // nz planes from z0 (the tile depth is a tuning parameter)
};

// A ghost cell: patch id and packed padded coordinates (i+3) | (j+3) << 10 | (k+3) << 20.
struct GhostRec {
  int32_t patch;
  uint32_t cell;
};

// One local patch's cover scan: the axis-aligned box of `ext` global cells around
// its bounding sphere of radius `radius`.
struct CoverJob {
  int32_t patch;
  int32_t ext[3];
  double radius;
};
// One workgroup of the cover scan: COVER_CPT x 256 consecutive cells of the
// box of one job, starting at cell `first` of that box.
#define COVER_CPT 4
struct CoverBlk {
  int32_t job;
  uint32_t first;
};

// A brick of ghost cells of one local patch: box [i0,i0+di) x [j0,j0+dj) x [k0,k0+dk)
// in interior-relative cell indices, at most BRICK_THREADS cells.
struct GBrick {
  int32_t patch, i0, j0, k0, di, dj, dk, pad;
};

// A ghost point that could not be interpolated: kind 0 = local ghost cell
// (packed padded coordinates), kind 1 = global effective ghost (linear index).
struct FallbackRec {
  int32_t patch, kind;
  uint32_t cell;
};

struct PostFlagsArgs {
  const uint8_t *flag;
  int32_t *efflist;
  int *effcount;
  uint8_t *dvalid[PW_NPTS];  // per interpolation width P = 2 .. 6 in use (else null)
  int Pvals[PW_NPTS];
  int donor_effghost;  // narrow buffer: effective ghosts count as valid donors
  uint8_t *t1, *t2;
  int n[3];
  int wrap[3];  // periodic axes of the global patch
};

struct L2GOrderArgs {
  const PatchDev *P;
  const PoseDev *pose;
  const int32_t *list;
  const int *count;
  const int32_t *cover;
  int nbuckets;
  int *cnt, *off, *ebkt, *erank;
  const int *rank;  // position of each bucket along its patch's Morton curve
  int32_t *sorted;  // entries grouped by bucket (scratch)
  int32_t *out;     // the same, ascending cell index within each bucket (may alias list)
  int2 *items;      // work items of the local -> global kernel: runs of <= L2G_ITEM entries of one bucket
  int *nitems;
};

struct FlagsArgs {
  const PatchDev *P;
  const PoseDev *pose;
  const CoverJob *jobs;
  const CoverBlk *blks;
  int njobs, nblks;
  // physical ghost cells of the global patch (outer ghosts that are not
  // periodic copies) and the list of those a local patch covers: entries
  // (index into phys, covering patch), count in *ocount
  const GhostRec *phys;
  int nphys;
  int2 *olist;
  int *ocount;
  int32_t *cover_new;
  uint8_t *t1, *t2, *live, *flag_new;
  uint8_t *dbl;  // cells claimed by two local patches
  int n[3];
  int wrap[3];   // periodic axes of the global patch
  int buffer;
  int *err;      // set if an overlap reaches a non-live cell
};

struct FinalizeArgs {
  const PatchDev *P;
  const PoseDev *pose;
  uint8_t *flag_cur;
  const uint8_t *flag_new;
  int32_t *cover_cur, *cover_new;
  int nsv;
  const int *Pts;
  const ExactDev *ex;
  const double *vs;
  const double *tdev;
  int mode;
  unsigned long long *counters;
  int n[3];
  int2 *ulist;  // cells that become live: (cell, previous cover id); capacity n0 n1 n2
  int *ucount;
  // covered physical ghosts of the global patch: the list of the next step
  // (olist_new) becomes the current one
  const int2 *olist_new;
  const int *ocount_new;
  int2 *olist_cur;
  int *ocount_cur;
  int nphys;
};

// Parts of a ghost fill: the global patch's (outer ghosts, effective ghosts)
// and the local patches' (periodic copies, interpatch bricks).
enum { GH_GLOBAL = 1, GH_LOCAL = 2 };
// Phases of one ghost fill (any subset, in this order): the interpatch kernels,
// the lower-priority value of their skipped points, the outer and periodic fill.
enum { PH_INTERP = 1, PH_FALLBACK = 2, PH_LOWER = 4, PH_ALL = 7 };

struct GhostArgs {
  const PatchDev *P;
  const PoseDev *pose;
  int parts;
  int phases;  // PH_* bits (the narrow-buffer order runs them all)
  // analytic outer ghosts of the global patch: the first midpoint stage also
  // writes them into the second one's buffer (lower_dup = that stage, else -1),
  // and the second skips them (lower_skip_global)
  int lower_dup, lower_skip_global;
  const GhostRec *lower;  // global-patch entries first, then local-patch entries
  int n_lower, n_lower_global;
  const GBrick *bricks;
  int n_bricks;
  const uint8_t *dvalid;
  const int32_t *efflist;  // effective ghosts grouped by donor bucket
  const int *effcount;
  const int2 *l2g_items;  // work items of the local -> global kernel (first entry, count)
  const int *l2g_nitems;
  const int32_t *cover;
  int has_locals;
  int gn[3];
  int sv, stage, stage_fp64, mixed, Pts;
  const ExactDev *ex;
  double v;
  const double *tdev;  // stage time = tdev[0] + tmul * dt
  double tmul, dt;
  unsigned long long *skips;
  FallbackRec *fb;  // capacity: every interpatch target of this part
  int *fb_count;
  int g2l_run, l2g_run;  // consecutive bricks / groups per XCD run
  int l2g_first;         // narrow buffer: local->global (and its fallbacks) before global->local
  int global_curv;       // curvilinear global patch: one-point-per-thread interpatch kernels
  int g2l_exact_only;    // the global patch does not carry sv and an exact solution is registered:
                         // the local ghosts take it directly (no donor, no fallback records)
  int l2g_direct;        // validation: every local->global point takes the direct gather
  const uint8_t *gflag;  // cover flags of the global patch (donor test of those kernels)
  // covered physical ghost cells of the global patch (Sec. 2.4.2): filled from
  // the covering local patch after their boundary value (null: none)
  const GhostRec *phys;
  const int2 *olist;
  const int *ocount;
  int nphys;  // physical ghost cells of the global patch (bound of the covered list)
};

struct StageArgs {
  const PatchDev *P;
  const PoseDev *pose;
  const TileRec *tiles;  // all of one topology (coord)
  int ntiles;
  int coord;
  int global;  // the tiles are those of the global patch (live-cell test applies)
  const uint8_t *gflag;
  int sv, stage, mixed;
  int inc;   // mixed path: FP32 increments in the accumulator
  int form;  // 0: the paper's Pi_t equation, 1: its first-order form
  int local_tile;   // tile shape of local patches (StageTile SH)
  int global_tile;  // tile shape of the global patch (StageTile SH)
  double dt, v2, eps;
};

void launch_pose(hipStream_t s, const PatchDev *P, int np, const double *tdev, double dt, PoseDev *poses);
void launch_pose_at(hipStream_t s, const PatchDev *P, int np, double t, PoseDev *out);
void launch_advance_time(hipStream_t s, double *tdev, double dt, long long *counters);
void launch_flags(hipStream_t s, const FlagsArgs &a);
void launch_finalize(hipStream_t s, const FinalizeArgs &a);
void launch_ghosts(hipStream_t s, const GhostArgs &a);
void launch_post_flags(hipStream_t s, const PostFlagsArgs &a);
void launch_l2g_order(hipStream_t s, const L2GOrderArgs &a);
void launch_stage(hipStream_t s, const StageArgs &a);
// Sommerfeld outer boundary: RK stage of the global patch's outer ghost cells
void launch_radiative(hipStream_t s, const PatchDev *P, const GhostRec *list, int count, int sv, int stage,
                      int mixed, int inc, double dt, double v);
// lower-priority fill (exact solution / nearest interior cell) of the listed
// cells of u (fp64 = 1) or of its FP32 copy (fp64 = 0) at time tdev[0]
void launch_fill_list(hipStream_t s, const PatchDev *P, const PoseDev *pose, const GhostRec *list, int count, int sv,
                      int fp64, const ExactDev *ex, double v, const double *tdev);
void launch_trig_table(hipStream_t s, int n1, int n2, double lo1, double dx1, double lo2, double dx2, double *tab);
void launch_fill_f64(hipStream_t s, double *p, long long n, double v);
void launch_fill_f32(hipStream_t s, float *p, long long n, float v);
void launch_fill_i32(hipStream_t s, int32_t *p, long long n, int32_t v);
void launch_fill_u8(hipStream_t s, uint8_t *p, long long n, uint8_t v);
void launch_unpack(hipStream_t s, const PatchDev *P, int pid, int sv, const double *src, long long n);
void launch_pack(hipStream_t s, const PatchDev *P, int pid, int sv, double *dst, long long n, int full);
void launch_init_exact(hipStream_t s, const PatchDev *P, const PoseDev *pose, int pid, int sv, const ExactDev *ex,
                       double v, double t, long long ncell);
void launch_diag(hipStream_t s, const PatchDev *P, const PoseDev *pose, int pid, int sv, const uint8_t *gflag,
                 const ExactDev *ex, double v, double t, double *partial, int nblocks);

}  // namespace pw
