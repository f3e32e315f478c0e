// HIP kernels of libpw for gfx950 (MI355X).
//
// One RK4 step of the multipatch scalar-wave system (arXiv 2002.00088):
//   pose      patch centres and velocities at the substep times      (Sec. 2.4.2)
//   flags     cover test, NG+1 live buffer, effective ghosts          (Sec. 2.4.2, Fig. cflag)
//   ghosts    analytic/periodic ghosts, then global->local and
//             local->global Lagrange interpolation with the frame
//             transform through the background frame                 (Secs. 2.4-2.4.2, Eq. Pijk)
//   stage     RHS of Eqs. eom1-eom3 + Kreiss-Oliger, RK4 stage update (Secs. 2.2-2.3, Table rk4)
//   finalize  flags at t_{n+1}, uncover fill, poison deactivated cells
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <initializer_list>
#include <type_traits>

#include "pw_internal.h"
#include "pw_kernels.h"

namespace pw {

// ---------------------------------------------------------------------------
// Pose: slot 0 = t_n, slot 1 = t_n + dt/2, slot 2 = t_n + dt (classic RK4
// abscissae c = 0, 1/2, 1/2, 1), slot 3 = an explicit time.
// ---------------------------------------------------------------------------
__global__ void k_pose(const PatchDev *P, int np, const double *tdev, double dt, PoseDev *poses) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double tn = tdev[0];
  pose_at(P[p], tn, poses[p]);
  pose_at(P[p], tn + 0.5 * dt, poses[np + p]);
  pose_at(P[p], tn + dt, poses[2 * np + p]);
}

__global__ void k_pose_at(const PatchDev *P, int np, double t, PoseDev *out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  pose_at(P[p], t, out[p]);
}

__global__ void k_advance_time(double *tdev, double dt, long long *counters) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    tdev[0] = tdev[0] + dt;
    counters[4] += 1;
  }
}

// ---------------------------------------------------------------------------
// Cover flags
// ---------------------------------------------------------------------------
// cover[c] = id of the local patch whose closed numerical box contains the
// centre of global cell c (Sec. 2.4.2: the covered test is done in the local
// patch's numerical coordinates).  Each local patch scans the global cells of
// the axis-aligned box around its bounding sphere (a Cartesian global), or all
// global cells (a curvilinear global: the host sets the extents to the grid).
// A cell claimed by two patches keeps the lower id and is marked in dbl.
__global__ __launch_bounds__(256) void k_cover(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose,
                                               const CoverJob *jobs, const CoverBlk *blks, int32_t *cover,
                                               uint8_t *dbl) {
  const CoverBlk B = blks[blockIdx.x];
  const CoverJob J = jobs[B.job];
  const PatchDev &g = P[0];
  const PatchDev &p = P[J.patch];
  const PoseDev &ps = pose[J.patch];
  int lo[3];
  for (int a = 0; a < 3; a++) {
    double c = (ps.c[a] - J.radius - g.lo[a]) * g.idx[a] - 0.5;
    c = c < -1.0e9 ? -1.0e9 : (c > 1.0e9 ? 1.0e9 : c);
    lo[a] = g.coord == CART ? (int)floor(c) : 0;
  }
  // the host keeps every box below 2^31 cells: 32-bit index arithmetic
  const unsigned e0 = (unsigned)J.ext[0], e1 = (unsigned)J.ext[1];
  const unsigned total = e0 * e1 * (unsigned)J.ext[2];
#pragma unroll
  for (int m = 0; m < COVER_CPT; m++) {
    const unsigned q = B.first + m * 256u + threadIdx.x;
    if (q >= total) break;
    const unsigned r = q / e0, kk = r / e1;
    const int i = lo[0] + (int)(q - r * e0);
    const int j = lo[1] + (int)(r - kk * e1);
    const int k = lo[2] + (int)kk;
    if (i < 0 || j < 0 || k < 0 || i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) continue;
    double X[3], xp[3];
    global_X(g, pose[0], i, j, k, X);
    const double d0 = X[0] - ps.c[0], d1 = X[1] - ps.c[1], d2 = X[2] - ps.c[2];
    if (d0 * d0 + d1 * d1 + d2 * d2 > J.radius * J.radius) continue;
    inv_map(p, ps, X, xp);
    bool in = true;
    for (int a = 0; a < 3; a++) {
      if (p.periodic[a]) continue;
      in = in && (xp[a] >= p.lo[a]) && (xp[a] <= p.hi[a]);
    }
    if (!in) continue;
    long long c = ((long long)k * g.n[1] + j) * g.n[0] + i;
    int old = atomicCAS(&cover[c], -1, J.patch);
    if (old != -1 && old != J.patch) {
      dbl[c] = 1;
      atomicMin(&cover[c], J.patch);
    }
  }
}

// Covered physical ghost cells of the global patch (Sec. 2.4.2, last
// paragraph): each outer ghost cell that is not a periodic copy is tested
// against the local patches in ascending id (the same closed-box test as
// k_cover); the first that contains its centre is recorded with it.
// Candidates first: with a Cartesian global only patches whose bounding
// sphere reaches past a face of the domain can cover an outer ghost centre;
// each workgroup lists them in LDS (ascending id) and exits if there are none.
#define COVER_OUTER_MAXJOBS 4096
__global__ __launch_bounds__(256) void k_cover_outer(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose,
                                                     const CoverJob *jobs, int njobs, const GhostRec *phys, int nphys,
                                                     int2 *olist, int *ocount) {
  __shared__ short cand[COVER_OUTER_MAXJOBS];
  __shared__ int ncand;
  __shared__ int wcnt[4];
  const PatchDev &g = P[0];
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  // one pass of 256 jobs at a time keeps the list in ascending id order
  for (int m0 = 0; m0 < njobs && m0 < COVER_OUTER_MAXJOBS; m0 += 256) {
    const int m = m0 + (int)threadIdx.x;
    bool c = false;
    if (m < njobs) {
      const CoverJob &J = jobs[m];
      const PoseDev &ps = pose[J.patch];
      c = g.coord != CART;
      for (int a = 0; a < 3 && !c; a++) c = ps.c[a] - J.radius < g.lo[a] || ps.c[a] + J.radius > g.hi[a];
    }
    const unsigned long long bal = __ballot(c);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) wcnt[wv] = __popcll(bal);
    __syncthreads();
    int base = ncand;
    for (int w = 0; w < wv; w++) base += wcnt[w];
    if (c) cand[base + __popcll(bal & ((1ull << lane) - 1ull))] = (short)m;
    __syncthreads();
    if (threadIdx.x == 0) ncand += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  const int nc = ncand;
  if (nc == 0) return;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nphys) return;
  int c[3];
  {
    const uint32_t w = phys[q].cell;
    c[0] = (int)(w & 1023u) - PW_NG;
    c[1] = (int)((w >> 10) & 1023u) - PW_NG;
    c[2] = (int)((w >> 20) & 1023u) - PW_NG;
  }
  double X[3];
  global_X(g, pose[0], c[0], c[1], c[2], X);
  for (int mc = 0; mc < nc; mc++) {
    const CoverJob &J = jobs[cand[mc]];
    const PatchDev &p = P[J.patch];
    const PoseDev &ps = pose[J.patch];
    const double d0 = X[0] - ps.c[0], d1 = X[1] - ps.c[1], d2 = X[2] - ps.c[2];
    if (d0 * d0 + d1 * d1 + d2 * d2 > J.radius * J.radius) continue;
    double xp[3];
    inv_map(p, ps, X, xp);
    bool in = true;
    for (int a = 0; a < 3; a++) {
      if (p.periodic[a]) continue;
      in = in && (xp[a] >= p.lo[a]) && (xp[a] <= p.hi[a]);
    }
    if (!in) continue;
    const int slot = atomicAdd(ocount, 1);
    olist[slot] = make_int2(q, J.patch);
    return;
  }
}

// Chebyshev dilation along one axis: out[c] = max_{|d|<=R} in[c + d e_axis],
// cells outside the domain read as `oob`.  With SRC_COVER the input is
// "uncovered" = (cover == -1).
template <int AXIS, bool SRC_COVER>
__global__ void k_dilate(const void *in_, uint8_t *out, int n0, int n1, int n2, int R, int oob, int wrap) {
  // grid (x blocks, n1, n2): no integer division for the cell coordinates
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= n0) return;
  const long long c = ((long long)k * n1 + j) * n0 + i;
  int pos = AXIS == 0 ? i : (AXIS == 1 ? j : k);
  int len = AXIS == 0 ? n0 : (AXIS == 1 ? n1 : n2);
  long long stride = AXIS == 0 ? 1 : (AXIS == 1 ? (long long)n0 : (long long)n0 * n1);
  int m = 0;
  for (int d = -R; d <= R; d++) {
    int q = pos + d;
    if (wrap) q = ((q % len) + len) % len;  // periodic axis of the global patch
    int v;
    if (q < 0 || q >= len) {
      v = oob;
    } else if (SRC_COVER) {
      v = ((const int32_t *)in_)[c + (long long)(q - pos) * stride] == -1;
    } else {
      v = ((const uint8_t *)in_)[c + (long long)(q - pos) * stride];
    }
    m = v > m ? v : m;
  }
  out[c] = (uint8_t)m;
}

// flag = live ? LIVE : (near a live cell ? EFFGHOST : DEACT)
// A cell covered by two local patches must stay live (overlap only in the
// buffers); otherwise the overlap error is raised.
__global__ void k_combine_flags(const uint8_t *live, const uint8_t *near, const uint8_t *dbl, uint8_t *flag,
                                long long total, int *err) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total) return;
  flag[c] = live[c] ? LIVE : (near[c] ? EFFGHOST : DEACT);
  if (dbl[c] && !live[c]) err[0] = 1;
}

// ---------------------------------------------------------------------------
// The same filters on 16-cell chunks (rows of a multiple of 16 cells, arrays
// 16-byte aligned): one thread per chunk, the chunk and its neighbours moved
// as 16-byte words.  Along x the cells of a 24-cell window become bits of a
// mask (radius <= 4); along y and z whole chunks of 0/1 bytes combine by OR
// (max) or AND (min).
// ---------------------------------------------------------------------------
static_assert(LIVE == 0 && EFFGHOST == 1 && DEACT == 2, "flag encoding used by the chunked filters");
// four bytes in {0, 1} -> four bits (byte m -> bit m)
__device__ __forceinline__ uint32_t bits4(uint32_t w) { return ((w * 0x01020408u) >> 24) & 0xFu; }
// four bits -> four bytes in {0, 1}
__device__ __forceinline__ uint32_t bytes4(uint32_t n) { return (n * 0x00204081u) & 0x01010101u; }
__device__ __forceinline__ uint32_t bits16(uint4 v) {
  return bits4(v.x) | (bits4(v.y) << 4) | (bits4(v.z) << 8) | (bits4(v.w) << 12);
}
__device__ __forceinline__ uint4 bytes16(uint32_t m) {
  return make_uint4(bytes4(m & 0xFu), bytes4((m >> 4) & 0xFu), bytes4((m >> 8) & 0xFu), bytes4((m >> 12) & 0xFu));
}
__device__ __forceinline__ uint32_t uncovered4(int4 v) {
  return (uint32_t)(v.x == -1) | ((uint32_t)(v.y == -1) << 1) | ((uint32_t)(v.z == -1) << 2) |
         ((uint32_t)(v.w == -1) << 3);
}
// chunk coordinates: grid (x blocks over the chunks of a plane, n2 planes)
struct Chunk {
  int ch, j, k, nch;
  long long row;  // first cell of the row
  bool ok;
};
__device__ __forceinline__ Chunk chunk_of(int n0, int n1) {
  Chunk q;
  q.nch = n0 >> 4;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  q.k = blockIdx.y;
  q.ok = t < (unsigned)(q.nch * n1);
  q.j = (int)(t / (unsigned)q.nch);
  q.ch = (int)t - q.j * q.nch;
  q.row = ((long long)q.k * n1 + q.j) * n0;
  return q;
}

// Dilation along x with radius R <= 4 (same result as k_dilate<0, SRC_COVER>).
template <bool SRC_COVER>
__global__ __launch_bounds__(256) void k_dilate_x16(const void *in_, uint8_t *out, int n0, int n1, int R, int oob,
                                                    int wrap) {
  const Chunk q = chunk_of(n0, n1);
  if (!q.ok) return;
  int chp = q.ch - 1, chn = q.ch + 1;
  bool hp = chp >= 0, hn = chn < q.nch;
  if (wrap) {
    if (!hp) chp = q.nch - 1;
    if (!hn) chn = 0;
    hp = hn = true;
  }
  const long long c = q.row + 16 * q.ch;
  uint32_t mid, pre = oob ? 0xFu : 0u, nxt = oob ? 0xFu : 0u;
  if (SRC_COVER) {
    const int32_t *in = (const int32_t *)in_;
    const int4 *v = (const int4 *)(in + c);
    mid = uncovered4(v[0]) | (uncovered4(v[1]) << 4) | (uncovered4(v[2]) << 8) | (uncovered4(v[3]) << 12);
    if (hp) pre = uncovered4(*(const int4 *)(in + q.row + 16 * chp + 12));
    if (hn) nxt = uncovered4(*(const int4 *)(in + q.row + 16 * chn));
  } else {
    const uint8_t *in = (const uint8_t *)in_;
    mid = bits16(*(const uint4 *)(in + c));
    if (hp) pre = bits4(*(const uint32_t *)(in + q.row + 16 * chp + 12));
    if (hn) nxt = bits4(*(const uint32_t *)(in + q.row + 16 * chn));
  }
  // bit t of M is cell x0 - 4 + t
  const uint32_t M = pre | (mid << 4) | (nxt << 20);
  uint32_t D = 0;
  for (int d = -R; d <= R; d++) D |= M >> (4 + d);
  *(uint4 *)(out + c) = bytes16(D & 0xFFFFu);
}

// Dilation along y (AXIS 1) or z (AXIS 2) of 0/1 bytes (k_dilate<AXIS, false>).
// With COMBINE the result is the "near a live cell" mask and the kernel writes
// the flags instead (k_combine_flags): flag = (1 - live) (2 - near) per byte.
template <int AXIS, bool COMBINE>
__global__ __launch_bounds__(256) void k_dilate_yz16(const uint8_t *in, uint8_t *out, int n0, int n1, int n2, int R,
                                                     int oob, int wrap, const uint8_t *live, const uint8_t *dbl,
                                                     int *err) {
  const Chunk q = chunk_of(n0, n1);
  if (!q.ok) return;
  const long long c = q.row + 16 * q.ch;
  const int pos = AXIS == 1 ? q.j : q.k, len = AXIS == 1 ? n1 : n2;
  const long long stride = AXIS == 1 ? (long long)n0 : (long long)n0 * n1;
  uint4 m = make_uint4(0, 0, 0, 0);
  for (int d = -R; d <= R; d++) {
    int p = pos + d;
    if (wrap) p = ((p % len) + len) % len;
    if (p < 0 || p >= len) {
      if (oob) m = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
    } else {
      const uint4 v = *(const uint4 *)(in + c + (long long)(p - pos) * stride);
      m.x |= v.x;
      m.y |= v.y;
      m.z |= v.z;
      m.w |= v.w;
    }
  }
  if (!COMBINE) {
    *(uint4 *)(out + c) = m;
    return;
  }
  const uint4 l = *(const uint4 *)(live + c), b = *(const uint4 *)(dbl + c);
  const uint4 nl = make_uint4(l.x ^ 0x01010101u, l.y ^ 0x01010101u, l.z ^ 0x01010101u, l.w ^ 0x01010101u);
  uint4 f;
  f.x = (0x02020202u - m.x) & (nl.x * 0xFFu);
  f.y = (0x02020202u - m.y) & (nl.y * 0xFFu);
  f.z = (0x02020202u - m.z) & (nl.z * 0xFFu);
  f.w = (0x02020202u - m.w) & (nl.w * 0xFFu);
  *(uint4 *)(out + c) = f;
  if ((b.x & nl.x) | (b.y & nl.y) | (b.z & nl.z) | (b.w & nl.w)) err[0] = 1;
}

// Forward window minimum along x, P <= 8 (k_window_min<0>): from the flags
// (from_flags 1: LIVE -> 1; 2: not DEACT -> 1) or from 0/1 bytes (0).
__device__ __forceinline__ uint32_t flagbits4(uint32_t w, int from_flags) {
  const uint32_t nw = ~w;
  const uint32_t b = from_flags == 1 ? (nw & (nw >> 1)) : (from_flags == 2 ? (nw >> 1) : w);
  return bits4(b & 0x01010101u);
}
__global__ __launch_bounds__(256) void k_window_x16(const uint8_t *in, uint8_t *out, int n0, int n1, int P,
                                                    int from_flags, int wrap) {
  const Chunk q = chunk_of(n0, n1);
  if (!q.ok) return;
  const long long c = q.row + 16 * q.ch;
  int chn = q.ch + 1;
  bool hn = chn < q.nch;
  if (wrap && !hn) {
    chn = 0;
    hn = true;
  }
  const uint4 v = *(const uint4 *)(in + c);
  uint32_t M = flagbits4(v.x, from_flags) | (flagbits4(v.y, from_flags) << 4) | (flagbits4(v.z, from_flags) << 8) |
               (flagbits4(v.w, from_flags) << 12);
  if (hn) {
    const uint2 w = *(const uint2 *)(in + q.row + 16 * chn);
    M |= (flagbits4(w.x, from_flags) << 16) | (flagbits4(w.y, from_flags) << 20);
  }
  uint32_t A = 0xFFFFFFFFu;
  for (int d = 0; d < P; d++) A &= M >> d;
  *(uint4 *)(out + c) = bytes16(A & 0xFFFFu);
}

// Forward window minimum along y (AXIS 1) or z (AXIS 2) of 0/1 bytes.
template <int AXIS>
__global__ __launch_bounds__(256) void k_window_yz16(const uint8_t *in, uint8_t *out, int n0, int n1, int n2, int P,
                                                     int wrap) {
  const Chunk q = chunk_of(n0, n1);
  if (!q.ok) return;
  const long long c = q.row + 16 * q.ch;
  const int pos = AXIS == 1 ? q.j : q.k, len = AXIS == 1 ? n1 : n2;
  const long long stride = AXIS == 1 ? (long long)n0 : (long long)n0 * n1;
  uint4 m = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
  for (int d = 0; d < P; d++) {
    int p = pos + d;
    if (wrap) p = p % len;
    if (p >= len) {
      m = make_uint4(0, 0, 0, 0);
    } else {
      const uint4 v = *(const uint4 *)(in + c + (long long)(p - pos) * stride);
      m.x &= v.x;
      m.y &= v.y;
      m.z &= v.z;
      m.w &= v.w;
    }
  }
  *(uint4 *)(out + c) = m;
}

// Tensor-product Lagrange interpolation of the 5 fields of buffer T of donor
// patch p at numerical point xd.  For a global donor every stencil cell must be
// live (gflag); for a local donor the stencil must lie in the interior (wrapping
// periodic axes).  Returns false if the point cannot be interpolated.
// The x-sums run in the compute type TC (x weights rounded to it); the outer
// sums over rows, with the FP64 weights wy[b] wz[c], in FP64.
template <typename TB, typename TC>
__device__ inline bool interp5(const PatchDev &p, const TB *T, const uint8_t *gflag, int P, const double xd[3],
                               double out[5], bool effghost_ok = false) {
  double wx[8], wy[8], wz[8];
  int s[3];
  double q[3];
  for (int a = 0; a < 3; a++) {
    q[a] = (xd[a] - p.lo[a]) * p.idx[a] - 0.5;
    if (!(q[a] > -1.0e6 && q[a] < 1.0e6)) return false;
  }
  s[0] = lagrange_w(P, q[0], wx);
  s[1] = lagrange_w(P, q[1], wy);
  s[2] = lagrange_w(P, q[2], wz);
  for (int a = 0; a < 3; a++)
    if (!p.periodic[a] && (s[a] < 0 || s[a] + P - 1 > p.n[a] - 1)) return false;
  if (p.is_global && gflag) {
    for (int c = 0; c < P; c++) {
      const int kk = p.periodic[2] ? ((s[2] + c) % p.n[2] + p.n[2]) % p.n[2] : s[2] + c;
      for (int b = 0; b < P; b++) {
        const int jj = p.periodic[1] ? ((s[1] + b) % p.n[1] + p.n[1]) % p.n[1] : s[1] + b;
        for (int a = 0; a < P; a++) {
          const int ii = p.periodic[0] ? ((s[0] + a) % p.n[0] + p.n[0]) % p.n[0] : s[0] + a;
          const uint8_t fl = gflag[((long long)kk * p.n[1] + jj) * p.n[0] + ii];
          if (effghost_ok ? fl == DEACT : fl != LIVE) return false;
        }
      }
    }
  }
  for (int f = 0; f < 5; f++) out[f] = 0.0;
  for (int c = 0; c < P; c++) {
    int kk = s[2] + c;
    if (p.periodic[2]) kk = ((kk % p.n[2]) + p.n[2]) % p.n[2];
    for (int b = 0; b < P; b++) {
      int jj = s[1] + b;
      if (p.periodic[1]) jj = ((jj % p.n[1]) + p.n[1]) % p.n[1];
      const double wyz = wy[b] * wz[c];
      TC part[5] = {0, 0, 0, 0, 0};
      for (int a = 0; a < P; a++) {
        int ii = s[0] + a;
        if (p.periodic[0]) ii = ((ii % p.n[0]) + p.n[0]) % p.n[0];
        long long x = cell_index(p, ii, jj, kk);
        TC w = (TC)wx[a];
        for (int f = 0; f < 5; f++) part[f] += w * (TC)T[f * p.fstride + x];
      }
      for (int f = 0; f < 5; f++) out[f] += wyz * (double)part[f];
    }
  }
  return true;
}

template <typename TB>
__device__ inline TB *stage_buf(const PatchDev &p, int sv, int stage) {
  // stage 1 reads u: FP64 in the FP64 path, its FP32 copy in the mixed path
  if (stage == 0) return sizeof(TB) == 8 ? (TB *)p.u[sv] : (TB *)p.us[sv];
  return (TB *)((stage == 2) ? p.vb[sv] : p.va[sv]);
}

// Interpolate donor d at background X, carry the result to receiver r at x_r.
template <typename TB, typename TC>
__device__ inline bool interp_transform(const PatchDev &d, const PoseDev &psd, const TB *T, const uint8_t *gflag,
                                        int P, const double X[3], const PatchDev &r, const PoseDev &psr,
                                        const double xr[3], double out[5]) {
  double xd[3];
  inv_map(d, psd, X, xd);
  double v[5];
  if (!interp5<TB, TC>(d, T, gflag, P, xd, v)) return false;
  double in4[4] = {(double)v[1], (double)v[2], (double)v[3], (double)v[4]}, G[3], pit, o4[4];
  patch_to_bg_at(d, psd, X, xd, in4, pit, G);
  bg_to_patch(r, psr, xr, pit, G, o4);
  out[0] = (double)v[0];
  for (int m = 0; m < 4; m++) out[1 + m] = o4[m];
  return true;
}

// Interpatch fills with a curvilinear global patch, one thread per point:
// the stencils gather straight from global memory (periodic axes wrap), so no
// donor box has to be contiguous in the global's index space.
// Global -> local: the ghost cells of the brick list.
template <typename TB, typename TC>
__global__ __launch_bounds__(BRICK_THREADS) void k_g2l_point(const PatchDev *__restrict__ P,
                                                             const PoseDev *__restrict__ pose, const GBrick *bricks,
                                                             int nbricks, int sv, int stage, const uint8_t *gflag,
                                                             int effghost_ok, int Pts, unsigned long long *skips,
                                                             FallbackRec *fb, int *fb_count) {
  const int bidx = blockIdx.x;
  if (bidx >= nbricks) return;
  const GBrick B = bricks[bidx];
  const PatchDev &r = P[B.patch];
  const PatchDev &G0 = P[0];
  const int tid = threadIdx.x;
  if (tid >= B.di * B.dj * B.dk) return;
  const int c[3] = {B.i0 + tid % B.di, B.j0 + (tid / B.di) % B.dj, B.k0 + tid / (B.di * B.dj)};
  bool inside = true, winside = true;
  for (int a = 0; a < 3; a++) {
    inside = inside && c[a] >= 0 && c[a] < r.n[a];
    const int w = r.periodic[a] ? ((c[a] % r.n[a]) + r.n[a]) % r.n[a] : c[a];
    winside = winside && w >= 0 && w < r.n[a];
  }
  if (!(r.sv_mask & (1u << sv)) || inside || winside) return;
  const bool has_donor = (G0.sv_mask & (1u << sv)) != 0;
  bool ok = false;
  double out[5];
  if (has_donor) {
    double X[3], xd[3];
    fwd_map_grid(r, pose[B.patch], c, X);
    inv_map(G0, pose[0], X, xd);
    double v[5];
    if (interp5<TB, TC>(G0, stage_buf<TB>(G0, sv, stage), gflag, Pts, xd, v, effghost_ok != 0)) {
      double in4[4] = {(double)v[1], (double)v[2], (double)v[3], (double)v[4]}, G[3], pit, o4[4];
      patch_to_bg(G0, pose[0], xd, in4, pit, G);
      bg_to_patch_grid(r, pose[B.patch], c, pit, G, o4);
      out[0] = (double)v[0];
      for (int m = 0; m < 4; m++) out[1 + m] = o4[m];
      ok = true;
    }
  }
  if (!ok) {
    if (has_donor) atomicAdd(skips, 1ull);
    const int slot = atomicAdd(fb_count, 1);
    fb[slot] = FallbackRec{B.patch, 0, (uint32_t)((c[0] + PW_NG) | ((c[1] + PW_NG) << 10) | ((c[2] + PW_NG) << 20))};
    return;
  }
  TB *TR = stage_buf<TB>(r, sv, stage);
  const long long dst = cell_index(r, c[0], c[1], c[2]);
  for (int f = 0; f < 5; f++) TR[f * r.fstride + dst] = (TB)out[f];
}

// Local -> global: the effective ghosts of the global patch.
template <typename TB, typename TC>
__global__ void k_l2g_point(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, const int32_t *list,
                            const int *count, const int32_t *cover, int sv, int stage, int Pts,
                            unsigned long long *skips, FallbackRec *fb, int *fb_count) {
  const PatchDev &G0 = P[0];
  if (!(G0.sv_mask & (1u << sv))) return;
  const int n = count[0];
  TB *TG = stage_buf<TB>(G0, sv, stage);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const long long c = list[q];
    const int i = (int)(c % G0.n[0]), j = (int)((c / G0.n[0]) % G0.n[1]),
              k = (int)(c / ((long long)G0.n[0] * G0.n[1]));
    const int d = cover[c];
    double out[5];
    bool ok = false;
    if (d >= 1 && (P[d].sv_mask & (1u << sv))) {
      const double xr[3] = {xnum(G0, 0, i), xnum(G0, 1, j), xnum(G0, 2, k)};
      double X[3];
      global_X(G0, pose[0], i, j, k, X);
      ok = interp_transform<TB, TC>(P[d], pose[d], stage_buf<TB>(P[d], sv, stage), nullptr, Pts, X, G0, pose[0], xr,
                                    out);
    }
    if (ok) {
      const long long dst = cell_index(G0, i, j, k);
      for (int f = 0; f < 5; f++) TG[f * G0.fstride + dst] = (TB)out[f];
    } else {
      atomicAdd(skips, 1ull);
      const int slot = atomicAdd(fb_count, 1);
      fb[slot] = FallbackRec{0, 1, (uint32_t)c};
    }
  }
}

__device__ inline void unpack_ijk(uint32_t c, int &i, int &j, int &k) {
  i = (int)(c & 1023u) - PW_NG;
  j = (int)((c >> 10) & 1023u) - PW_NG;
  k = (int)((c >> 20) & 1023u) - PW_NG;
}

// Local -> global into the covered physical ghost cells of the global patch
// (Sec. 2.4.2, last paragraph), after their boundary value: a point whose
// stencil leaves the donor's interior keeps that value (counted in
// counters[5]); counters[6] counts the targets.
template <typename TB, typename TC>
__global__ void k_l2g_outer(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, const GhostRec *phys,
                            const int2 *olist, const int *ocount, int sv, int stage, int Pts,
                            unsigned long long *counters) {
  const PatchDev &G0 = P[0];
  if (!(G0.sv_mask & (1u << sv))) return;
  const int n = ocount[0];
  TB *TG = stage_buf<TB>(G0, sv, stage);
  unsigned sk = 0;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int2 e = olist[q];
    int i, j, k;
    unpack_ijk(phys[e.x].cell, i, j, k);
    const int d = e.y;
    double out[5];
    bool ok = false;
    if (P[d].sv_mask & (1u << sv)) {
      const double xr[3] = {xnum(G0, 0, i), xnum(G0, 1, j), xnum(G0, 2, k)};
      double X[3];
      global_X(G0, pose[0], i, j, k, X);
      ok = interp_transform<TB, TC>(P[d], pose[d], stage_buf<TB>(P[d], sv, stage), nullptr, Pts, X, G0, pose[0], xr,
                                    out);
    }
    if (ok) {
      const long long dst = cell_index(G0, i, j, k);
      for (int f = 0; f < 5; f++) TG[f * G0.fstride + dst] = (TB)out[f];
    } else {
      sk++;
    }
  }
  if (sk) atomicAdd(&counters[5], (unsigned long long)sk);
  if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) atomicAdd(&counters[6], (unsigned long long)n);
}

// The covered-ghost list of the next step becomes the current one.
__global__ void k_copy_olist(const int2 *src, const int *nsrc, int2 *dst, int *ndst) {
  const int n = nsrc[0];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) dst[q] = src[q];
  if (blockIdx.x == 0 && threadIdx.x == 0) ndst[0] = n;
}

// Lower-priority ghost data: periodic copy if the wrapped index is interior,
// else the exact solution (analytic outer boundary) or the nearest interior cell.
template <typename TB>
__global__ void k_fill_lower(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, const GhostRec *list, int count, int sv, int stage,
                             const ExactDev *ex, double v, const double *tdev, double tmul, double dt, int stage2) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const double t = tdev[0] + tmul * dt;
  GhostRec g = list[q];
  const PatchDev &p = P[g.patch];
  if (!(p.sv_mask & (1u << sv))) return;
  TB *T = stage_buf<TB>(p, sv, stage);
  int c[3];
  unpack_ijk(g.cell, c[0], c[1], c[2]);
  int w[3];
  bool interior = true;
  for (int a = 0; a < 3; a++) {
    w[a] = c[a];
    if (p.periodic[a]) w[a] = ((c[a] % p.n[a]) + p.n[a]) % p.n[a];
    interior = interior && w[a] >= 0 && w[a] < p.n[a];
  }
  long long dst = cell_index(p, c[0], c[1], c[2]);
  if (interior) {
    long long src = cell_index(p, w[0], w[1], w[2]);
    for (int f = 0; f < 5; f++) T[f * p.fstride + dst] = T[f * p.fstride + src];
  } else if (ex[sv].kind != EX_NONE) {
    double xp[3] = {xnum(p, 0, c[0]), xnum(p, 1, c[1]), xnum(p, 2, c[2])}, e[5];
    exact_patch(ex[sv], v, p, pose[g.patch], t, xp, e);
    for (int f = 0; f < 5; f++) T[f * p.fstride + dst] = (TB)e[f];
    if (stage2 >= 0) {
      // a second stage at the same time (the two midpoint stages) gets the same values
      TB *T2 = stage_buf<TB>(p, sv, stage2);
      for (int f = 0; f < 5; f++) T2[f * p.fstride + dst] = (TB)e[f];
    }
  } else {
    for (int a = 0; a < 3; a++) w[a] = w[a] < 0 ? 0 : (w[a] >= p.n[a] ? p.n[a] - 1 : w[a]);
    long long src = cell_index(p, w[0], w[1], w[2]);
    for (int f = 0; f < 5; f++) T[f * p.fstride + dst] = T[f * p.fstride + src];
  }
}

// ---------------------------------------------------------------------------
// Per-step helper arrays of the global patch
// ---------------------------------------------------------------------------
// Forward window minimum along one axis: out[c] = min_{0<=d<P} in[c + d e_axis],
// cells beyond the domain read 0.  Applied along x (from the flags, LIVE -> 1),
// y and z it gives dvalid[c] = 1 iff the P^3 donor box starting at c is all live.
template <int AXIS>
__global__ void k_window_min(const uint8_t *in, uint8_t *out, int n0, int n1, int n2, int P, int from_flags,
                             int wrap) {
  // grid (x blocks, n1, n2): no integer division for the cell coordinates
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= n0) return;
  const long long c = ((long long)k * n1 + j) * n0 + i;
  int pos = AXIS == 0 ? i : (AXIS == 1 ? j : k);
  int len = AXIS == 0 ? n0 : (AXIS == 1 ? n1 : n2);
  long long stride = AXIS == 0 ? 1 : (AXIS == 1 ? (long long)n0 : (long long)n0 * n1);
  int m = 1;
  for (int d = 0; d < P; d++) {
    int v = 0;
    int q = pos + d;
    if (wrap) q = q % len;  // periodic axis of the global patch
    if (q < len) {
      const uint8_t x = in[c + (long long)(q - pos) * stride];
      v = from_flags == 1 ? (x == LIVE) : (from_flags == 2 ? (x != DEACT) : x);
    }
    m = v < m ? v : m;
  }
  out[c] = (uint8_t)m;
}

__global__ void k_set_int(int *p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

// Compacted list of the effective ghost cells.  Cells are visited in 4x4x4
// brick order, so consecutive list entries are 3-D neighbours whose donor
// stencils overlap (cache reuse in the local->global gather).  One atomic per
// workgroup of 256 x EFF_PER_THREAD cells; the order of the list does not affect
// any result.
#define EFF_PER_THREAD 16
__global__ __launch_bounds__(256) void k_efflist(const uint8_t *flag, int n0, int n1, int n2, int32_t *list,
                                                 int *count) {
  __shared__ int wsum[4], wbase[4], bbase;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nbx = (n0 + 3) >> 2, nby = (n1 + 3) >> 2, nbz = (n2 + 3) >> 2;
  const long long total = (long long)nbx * nby * nbz * 64;
  const long long start = (long long)blockIdx.x * 256 * EFF_PER_THREAD;
  unsigned long long masks[EFF_PER_THREAD];
  int32_t cells[EFF_PER_THREAD];
  int mine = 0;
#pragma unroll
  for (int r = 0; r < EFF_PER_THREAD; r++) {
    const long long L = start + (long long)r * 256 + threadIdx.x;
    bool e = false;
    int32_t c = 0;
    if (L < total) {
      const long long b = L >> 6;
      const int q = (int)(L & 63);
      const int i = (int)(b % nbx) * 4 + (q & 3);
      const int j = (int)((b / nbx) % nby) * 4 + ((q >> 2) & 3);
      const int k = (int)(b / ((long long)nbx * nby)) * 4 + (q >> 4);
      if (i < n0 && j < n1 && k < n2) {
        c = (int32_t)(((long long)k * n1 + j) * n0 + i);
        e = flag[c] == EFFGHOST;
      }
    }
    cells[r] = c;
    masks[r] = __ballot(e);
    mine += (int)__popcll(masks[r]);
  }
  if (lane == 0) wsum[w] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    bbase = tot ? atomicAdd(count, tot) : 0;
    int acc = 0;
    for (int q = 0; q < 4; q++) { wbase[q] = acc; acc += wsum[q]; }
  }
  __syncthreads();
  int off = bbase + wbase[w];
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < EFF_PER_THREAD; r++) {
    if ((masks[r] >> lane) & 1ull) list[off + __popcll(masks[r] & below)] = cells[r];
    off += (int)__popcll(masks[r]);
  }
}

// Ordering of the effective ghosts by donor position: a counting sort by
// (covering local patch, 8 x 8 x 4-cell bucket of that patch holding the
// point), so that the points of a local -> global work item share one donor
// box.
__global__ void k_bucket_count(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, const int32_t *list, const int *count,
                               const int32_t *cover, const int *rank, int *cnt, int *ebkt, int *erank) {
  const PatchDev &G0 = P[0];
  const int n = count[0];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int stride = gridDim.x * blockDim.x;
  // whole wavefronts step through the list together (the ballots below need
  // every lane)
  for (int q0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63); q0 < n; q0 += stride) {
    const int q = q0 + lane;
    const bool act = q < n;
    int b = 0;
    if (act) {
      const long long c = list[q];
      const int i = (int)(c % G0.n[0]), j = (int)((c / G0.n[0]) % G0.n[1]),
                k = (int)(c / ((long long)G0.n[0] * G0.n[1]));
      const int d = cover[c];
      if (d >= 1) {
        const PatchDev &D = P[d];
        double X[3], xd[3];
        global_X(G0, pose[0], i, j, k, X);
        inv_map(D, pose[d], X, xd);
        int bi[3];
        for (int a = 0; a < 3; a++) {
          double qq = (xd[a] - D.lo[a]) * D.idx[a];
          int ii = (qq > -1.0e6 && qq < 1.0e6) ? (int)floor(qq) : 0;
          if (D.periodic[a]) ii = ((ii % D.n[a]) + D.n[a]) % D.n[a];
          ii = ii < 0 ? 0 : (ii >= D.n[a] ? D.n[a] - 1 : ii);
          bi[a] = ii >> (a == 2 ? 2 : 3);
        }
        b = D.bkt_base + rank[D.bkt_base + (bi[2] * D.bkt_n[1] + bi[1]) * D.bkt_n[0] + bi[0]];
      }
      ebkt[q] = b;
    }
    // neighbouring entries mostly share a bucket: one atomic per distinct bucket
    // of the wavefront, the lanes ranked in lane order behind its old count
    unsigned long long todo = __ballot(act);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int lb = __shfl(b, leader);
      const unsigned long long same = __ballot(act && b == lb) & todo;
      int base = 0;
      if (lane == leader) base = atomicAdd(&cnt[lb], __popcll(same));
      base = __shfl(base, leader);
      if ((same >> lane) & 1ull) erank[q] = base + __popcll(same & below);
      todo &= ~same;
    }
  }
}

// Exclusive scan of nb bucket counts by one workgroup of 1024 threads, in
// tiles of 8192 counts: thread t takes counts 8t .. 8t + 7 of a tile (a
// wavefront reads one contiguous 2 KB piece), the thread sums of the tile are
// scanned by wavefront shuffles and then across the 16 wavefront totals in LDS,
// and a running total carries from one tile to the next.
__global__ __launch_bounds__(1024) void k_bucket_scan(const int *cnt, int *off, int nb) {
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int carry = 0;  // the same in every thread
  for (int base = 0; base < nb; base += 8 * 1024) {
    const int b0 = base + 8 * t;
    int v[8];
#pragma unroll
    for (int m = 0; m < 8; m++) v[m] = b0 + m < nb ? cnt[b0 + m] : 0;
    int s = 0;
#pragma unroll
    for (int m = 0; m < 8; m++) s += v[m];
    int x = s;  // inclusive scan of the thread sums over the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const int ws = wsum[q];
      wpre += q < w ? ws : 0;
      tot += ws;
    }
    int run = carry + wpre + (x - s);  // counts before this thread's first bucket
#pragma unroll
    for (int m = 0; m < 8; m++)
      if (b0 + m < nb) {
        off[b0 + m] = run;
        run += v[m];
      }
    carry += tot;
    __syncthreads();  // wsum is written again by the next tile
  }
}

__global__ void k_bucket_scatter(const int32_t *list, const int *count, const int *ebkt, const int *erank,
                                 const int *off, int32_t *sorted) {
  const int n = count[0];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
    sorted[off[ebkt[q]] + erank[q]] = list[q];
}

// Each bucket's entries in ascending global cell index (rank by counting; one
// workgroup per bucket, keys staged in LDS when they fit).  The list order, and
// so the grouping of the local->global kernel, is then independent of the order
// in which the atomics of the bucket count were served.
__global__ __launch_bounds__(256) void k_bucket_sort(const int32_t *in, const int *cnt, const int *off, int nb,
                                                     int32_t *out) {
  __shared__ int32_t keys[BUCKET_SORT_LDS];
  const int b = blockIdx.x;
  if (b >= nb) return;
  const int m = cnt[b];
  if (m == 0) return;
  const int o = off[b];
  const int32_t *src = in + o;
  if (m > BUCKET_SORT_LDS) {
    // a bucket larger than the LDS tile keeps the scatter order (the order of
    // the list affects no value, only the locality of the gathers)
    for (int t = threadIdx.x; t < m; t += blockDim.x) out[o + t] = src[t];
    return;
  }
  // bitonic sort of the bucket's cell indices (unique) in LDS, padded to a power of two
  int m2 = 1;
  while (m2 < m) m2 <<= 1;
  for (int t = threadIdx.x; t < m2; t += blockDim.x) keys[t] = t < m ? src[t] : INT32_MAX;
  __syncthreads();
  for (int k = 2; k <= m2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < m2; t += blockDim.x) {
        const int u = t ^ j;
        if (u > t) {
          const int32_t x = keys[t], y = keys[u];
          if ((x > y) == ((t & k) == 0)) {
            keys[t] = y;
            keys[u] = x;
          }
        }
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < m; t += blockDim.x) out[o + t] = keys[t];
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).  Map
// workgroup v to a work item so that every XCD receives runs of K consecutive
// items: item = ((j / K) * 8 + x) * K + j % K with x = v mod 8, j = v / 8.  A
// bijection of [0, 8 K m) for every m.
__device__ __forceinline__ int xcd_spread(int v, int K) {
  const int x = v & 7, j = v >> 3;
  return ((j / K) * 8 + x) * K + (j % K);
}

// ---------------------------------------------------------------------------
// Global -> local (Sec. 2.4.1).  One workgroup per brick of up to 8x8x3 ghost
// cells of one face of a local patch.  Each thread locates its point in the
// global patch (FP64) and forms its Lagrange weights (FP64); the union of the
// donor stencils (the donor box) is staged in LDS and every thread sums its P^3
// taps from LDS.  FP32 sums: one float4 (fields 0-3) and one float (field 4)
// per box cell, staged in chunks of whole z-layers, so a tap is one 128-bit LDS
// read plus half of a two-dword read, and the taps of a row are immediate
// offsets from one row address; 30 KB of LDS and at most 128 VGPRs keep four
// waves per SIMD.  FP64 sums: the box field after field.  Validity is one
// byte: every cell of the donor stencil must be live.  Points that cannot be
// interpolated keep the lower-priority value (analytic or nearest interior)
// and are counted.
// ---------------------------------------------------------------------------
template <typename TB, typename TC, int Pts>
__global__ __launch_bounds__(BRICK_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_g2l_brick(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose,
                                                             const GBrick *bricks, int nbricks, int run, int sv,
                                                             int stage, const uint8_t *dvalid,
                                                             unsigned long long *skips, FallbackRec *fb,
                                                             int *fb_count) {
  // FP32 sums: the donor box as one float4 (fields 0-3) plus one float (field
  // 4) per cell, 20 bytes a cell, so a tap is one 128-bit LDS read and half of a
  // two-dword read; FP64 sums: field after field
  constexpr bool VEC = sizeof(TC) == 4;
  constexpr int INFLIGHT = 4;  // box cells per thread with their loads in flight together
  typedef double TO;           // type of the outer (y, z) sums: FP64 weights, FP64 accumulation
  constexpr int CAPV = BRICK_LDS_BYTES / 20;  // cells of a float4 + float box
  __shared__ __align__(16) unsigned char lds_raw[BRICK_LDS_BYTES];
  constexpr int NWAVE = BRICK_THREADS / 64;
  __shared__ int wbox[NWAVE][6];  // per wavefront: lowest and highest donor index per axis
  // runs of `run` consecutive bricks (which share donor cells) on one XCD
  const int bidx = xcd_spread(blockIdx.x, run);
  if (bidx >= nbricks) return;
  const GBrick B = bricks[bidx];
  const PatchDev &r = P[B.patch];
  const PatchDev &G0 = P[0];
  const int tid = threadIdx.x;
  const int c[3] = {B.i0 + tid % B.di, B.j0 + (tid / B.di) % B.dj, B.k0 + tid / (B.di * B.dj)};
  bool active = tid < B.di * B.dj * B.dk;
  if (active) {
    bool inside = true, winside = true;
    for (int a = 0; a < 3; a++) {
      inside = inside && c[a] >= 0 && c[a] < r.n[a];
      int w = r.periodic[a] ? ((c[a] % r.n[a]) + r.n[a]) % r.n[a] : c[a];
      winside = winside && w >= 0 && w < r.n[a];
    }
    active = (r.sv_mask & (1u << sv)) && !inside && !winside;
  }
  const bool has_donor = (G0.sv_mask & (1u << sv)) != 0;
  bool valid = false;
  int s[3] = {0, 0, 0};
  double wx[Pts], wy[Pts], wz[Pts];
  double xd[3] = {0, 0, 0};
  if (active && has_donor) {
    // background position; the global patch's numerical coordinates are X itself
    fwd_map_grid(r, pose[B.patch], c, xd);
    double q[3];
    bool fin = true;
    for (int a = 0; a < 3; a++) {
      q[a] = (xd[a] - G0.lo[a]) * G0.idx[a] - 0.5;
      fin = fin && (q[a] > -1.0e6 && q[a] < 1.0e6);
    }
    if (fin) {
      s[0] = lagrange_wt<Pts>(q[0], wx);
      s[1] = lagrange_wt<Pts>(q[1], wy);
      s[2] = lagrange_wt<Pts>(q[2], wz);
      bool inr = true;
      for (int a = 0; a < 3; a++) inr = inr && s[a] >= 0 && s[a] + Pts - 1 <= G0.n[a] - 1;
      if (inr) valid = dvalid[((long long)s[2] * G0.n[1] + s[1]) * G0.n[0] + s[0]] != 0;
    }
  }
  // the donor box: the union of the valid points' stencils, reduced within each
  // wavefront by xor shuffles, the wavefronts' boxes combined through LDS
  // (contended LDS atomics on six words cost more than the interpolation sums)
  {
    int bl[3], bh[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      bl[a] = valid ? s[a] : (1 << 30);
      bh[a] = valid ? s[a] + Pts - 1 : -(1 << 30);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int a = 0; a < 3; a++) {
        bl[a] = min(bl[a], __shfl_xor(bl[a], off));
        bh[a] = max(bh[a], __shfl_xor(bh[a], off));
      }
    if ((tid & 63) == 0)
#pragma unroll
      for (int a = 0; a < 3; a++) {
        wbox[tid >> 6][a] = bl[a];
        wbox[tid >> 6][3 + a] = bh[a];
      }
  }
  __syncthreads();
  int blo[3], bhi[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    blo[a] = wbox[0][a];
    bhi[a] = wbox[0][3 + a];
#pragma unroll
    for (int w = 1; w < NWAVE; w++) {
      blo[a] = min(blo[a], wbox[w][a]);
      bhi[a] = max(bhi[a], wbox[w][3 + a]);
    }
  }
  const int lo0 = blo[0], lo1 = blo[1], lo2 = blo[2];
  const int e0 = bhi[0] - lo0 + 1, e1 = bhi[1] - lo1 + 1, e2 = bhi[2] - lo2 + 1;
  const long long vol = (e0 > 0 && e1 > 0 && e2 > 0) ? (long long)e0 * e1 * e2 : 0;
  const TB *T = stage_buf<TB>(G0, sv, stage);
  // the x-row sums run in the compute type with the x weights rounded to it
  // once; the row sums are combined with the FP64 products wy[b] wz[c] in FP64
  TO acc[5] = {0, 0, 0, 0, 0};
  TC wxc[Pts];
#pragma unroll
  for (int a = 0; a < Pts; a++) wxc[a] = (TC)wx[a];
  const uint32_t gfs = (uint32_t)G0.fstride, gsy = (uint32_t)G0.pitch, gsz = (uint32_t)G0.slab;
  const int e01 = e0 * e1;
  bool staged = false;
  if constexpr (VEC) {
    // z-chunks of whole layers, all five fields at once
    float4 *box4 = (float4 *)lds_raw;
    float *box1 = (float *)(lds_raw + 16 * CAPV);
    const int nzc = e01 > 0 ? CAPV / e01 : 0;
    if (vol > 0 && nzc > 0) {
      staged = true;
      const float ie0 = 1.0f / (float)e0, ie1 = 1.0f / (float)e1;
      for (int z0 = 0; z0 < e2; z0 += nzc) {
        const int nz = e2 - z0 < nzc ? e2 - z0 : nzc;
        const int v = e01 * nz;
        const uint32_t base0 =
            (uint32_t)(lo0 + PW_OX) + (uint32_t)(lo1 + PW_NG) * gsy + (uint32_t)(lo2 + z0 + PW_NG) * gsz;
        // flat index q -> (x, row), row -> (b, layer) with float reciprocals:
        // exact, since (q + 0.5) / e lies at least 1/(2e) from an integer, q < 2^14
        for (int q0 = tid; q0 < v; q0 += INFLIGHT * BRICK_THREADS) {
          float tmp[INFLIGHT][5];
#pragma unroll
          for (int m = 0; m < INFLIGHT; m++) {
            const int q = q0 + m * BRICK_THREADS;
            if (q < v) {
              const int row = (int)(((float)q + 0.5f) * ie0);
              const int x = q - row * e0;
              const int cc = (int)(((float)row + 0.5f) * ie1);
              const int b = row - cc * e1;
              const uint32_t g = base0 + (uint32_t)b * gsy + (uint32_t)cc * gsz + (uint32_t)x;
#pragma unroll
              for (int f = 0; f < 5; f++) tmp[m][f] = (float)gld(T, (uint32_t)f * gfs + g);
            }
          }
#pragma unroll
          for (int m = 0; m < INFLIGHT; m++) {
            const int q = q0 + m * BRICK_THREADS;
            if (q < v) {
              box4[q] = make_float4(tmp[m][0], tmp[m][1], tmp[m][2], tmp[m][3]);
              box1[q] = tmp[m][4];
            }
          }
        }
        __syncthreads();
        if (valid) {
          // row pointers advance by e0 cells per row and e01 per layer, so every
          // tap of a row is an immediate offset from one address
          const int first = (s[2] - lo2 - z0) * e01 + (s[1] - lo1) * e0 + (s[0] - lo0);
          const float4 *r4 = box4 + first;
          const float *r1 = box1 + first;
          const int skip = e01 - Pts * e0;  // from the end of one layer's rows to the next layer
#pragma unroll
          for (int cc = 0; cc < Pts; cc++) {
            const int lz = s[2] - lo2 + cc - z0;  // layer of the chunk
            if (lz < 0 || lz >= nz) {
              r4 += e01;
              r1 += e01;
              continue;
            }
            // the layer's rows combined with the FP64 y weights, the layers
            // with the FP64 z weights
            TO ly[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int b = 0; b < Pts; b++) {
              float4 w4[Pts];
              float w1[Pts];
#pragma unroll
              for (int a = 0; a < Pts; a++) {
                w4[a] = r4[a];
                w1[a] = r1[a];
              }
              r4 += e0;
              r1 += e0;
              float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f;
#pragma unroll
              for (int a = 0; a < Pts; a++) {
                p0 += wxc[a] * w4[a].x;
                p1 += wxc[a] * w4[a].y;
                p2 += wxc[a] * w4[a].z;
                p3 += wxc[a] * w4[a].w;
                p4 += wxc[a] * w1[a];
              }
              const TO wb = (TO)wy[b];
              ly[0] += wb * (TO)p0;
              ly[1] += wb * (TO)p1;
              ly[2] += wb * (TO)p2;
              ly[3] += wb * (TO)p3;
              ly[4] += wb * (TO)p4;
            }
#pragma unroll
            for (int f = 0; f < 5; f++) acc[f] += (TO)wz[cc] * ly[f];
            r4 += skip;
            r1 += skip;
          }
        }
        if (z0 + nzc < e2) __syncthreads();
      }
    }
  } else {
    // FP64: as many fields per pass as fit, field after field
    TC *box = (TC *)lds_raw;
    constexpr int CAP = BRICK_LDS_BYTES / sizeof(TC);
    const int nfp = vol > 0 ? (int)(CAP / vol < 5 ? CAP / vol : 5) : 0;  // fields per LDS pass
    if (nfp > 0) {
      staged = true;
      const int v = (int)vol;
      const uint32_t base0 = (uint32_t)(lo0 + PW_OX) + (uint32_t)(lo1 + PW_NG) * gsy + (uint32_t)(lo2 + PW_NG) * gsz;
      const float ie0 = 1.0f / (float)e0, ie1 = 1.0f / (float)e1;
      for (int f0 = 0; f0 < 5; f0 += nfp) {
        const int nf = 5 - f0 < nfp ? 5 - f0 : nfp;
        for (int q0 = tid; q0 < v; q0 += 4 * BRICK_THREADS) {
          TC tmp[4][5];
#pragma unroll
          for (int m = 0; m < 4; m++) {
            const int q = q0 + m * BRICK_THREADS;
            if (q < v) {
              const int row = (int)(((float)q + 0.5f) * ie0);
              const int x = q - row * e0;
              const int cc = (int)(((float)row + 0.5f) * ie1);
              const int b = row - cc * e1;
              const uint32_t g = base0 + (uint32_t)b * gsy + (uint32_t)cc * gsz + (uint32_t)x;
#pragma unroll
              for (int f = 0; f < 5; f++)
                if (f < nf) tmp[m][f] = (TC)gld(T, (uint32_t)(f0 + f) * gfs + g);
            }
          }
#pragma unroll
          for (int m = 0; m < 4; m++) {
            const int q = q0 + m * BRICK_THREADS;
            if (q < v) {
#pragma unroll
              for (int f = 0; f < 5; f++)
                if (f < nf) box[f * v + q] = tmp[m][f];
            }
          }
        }
        __syncthreads();
        if (valid) {
          const TC *base = box + (s[2] - lo2) * e01 + (s[1] - lo1) * e0 + (s[0] - lo0);
          for (int f = 0; f < nf; f++) {
            TO sum = (TO)0;
            const TC *bf = base + f * v;
#pragma unroll
            for (int cc = 0; cc < Pts; cc++) {
              // row by row (a whole layer held in registers, 2 P^2 VGPRs in
              // FP64, spilled to scratch memory)
#pragma unroll
              for (int b = 0; b < Pts; b++) {
                TC w[Pts];
#pragma unroll
                for (int a = 0; a < Pts; a++) w[a] = bf[cc * e01 + b * e0 + a];
                TC part = (TC)0;
#pragma unroll
                for (int a = 0; a < Pts; a++) part += wxc[a] * w[a];
                sum += (TO)(wy[b] * wz[cc]) * (TO)part;
              }
            }
#pragma unroll
            for (int m = 0; m < 5; m++)
              if (m == f0 + f) acc[m] = sum;
          }
        }
        if (f0 + nfp < 5) __syncthreads();
      }
    }
  }
  if (!staged && valid) {
    // donor box larger than the LDS tile: gather straight from global memory
    // (weights picked by selects, so no array is indexed dynamically)
    for (int cc = 0; cc < Pts; cc++) {
      double wzd = 0.0;
#pragma unroll
      for (int m = 0; m < Pts; m++) wzd = (m == cc) ? wz[m] : wzd;
      for (int b = 0; b < Pts; b++) {
        double wyd = 0.0;
#pragma unroll
        for (int m = 0; m < Pts; m++) wyd = (m == b) ? wy[m] : wyd;
        TC part[5] = {0, 0, 0, 0, 0};
        const uint32_t x0 = (uint32_t)cell_index(G0, s[0], s[1] + b, s[2] + cc);
#pragma unroll
        for (int a = 0; a < Pts; a++)
#pragma unroll
          for (int f = 0; f < 5; f++) part[f] += wxc[a] * (TC)gld(T, f * gfs + x0 + a);
        const TO wyz = (TO)(wyd * wzd);
#pragma unroll
        for (int f = 0; f < 5; f++) acc[f] += wyz * (TO)part[f];
      }
    }
  }
  if (!active) return;
  if (!valid) {
    // rare: handled by k_fallback (lower-priority value, counted if a donor exists)
    if (has_donor) atomicAdd(skips, 1ull);
    const int slot = atomicAdd(fb_count, 1);
    fb[slot] = FallbackRec{B.patch, 0, (uint32_t)((c[0] + PW_NG) | ((c[1] + PW_NG) << 10) | ((c[2] + PW_NG) << 20))};
    return;
  }
  double out[5];
  {
    // the global patch's numerical frame is the background frame (Cartesian,
    // static, unrotated): its one-form needs no transformation
    const double G[3] = {(double)acc[2], (double)acc[3], (double)acc[4]};
    double o4[4];
    bg_to_patch_grid(r, pose[B.patch], c, (double)acc[1], G, o4);
    out[0] = (double)acc[0];
    for (int m = 0; m < 4; m++) out[1 + m] = o4[m];
  }
  TB *TR = stage_buf<TB>(r, sv, stage);
  long long dst = cell_index(r, c[0], c[1], c[2]);
  for (int f = 0; f < 5; f++) TR[f * r.fstride + dst] = (TB)out[f];
}

// ---------------------------------------------------------------------------
// Local -> global (Sec. 2.4.2).  The effective ghost cells are sorted by the
// donor bucket (8 x 8 x 4 cells of the covering local patch) that holds their
// donor point, and each bucket is cut into work items of at most L2G_ITEM
// consecutive entries (k_l2g_items).  The donor stencils of an item's points
// start within its bucket, so their union (the donor box) spans at most
// 14 x 14 x 10 cells (P = 6) and is staged in LDS once, all five fields per
// cell.  Each point is summed by K threads (K = 3, or 6 for items of at most
// 32 points), thread g of a point taking its z-layers g, g + K, ...; the layer
// sums l_c meet as (l_0 + l_3) + (l_1 + l_4) + (l_2 + l_5) whatever K is, so a
// point's value does not depend on how the list was cut.  The x-row sums run
// in the compute type with the x weights rounded to it, the y and z sums in
// FP64 with FP64 weights (explicit FMAs and roundings, so the staged and the
// direct path below agree bitwise).  Points whose box does not fit the LDS
// tile gather their stencil from global memory with the same arithmetic.
// ---------------------------------------------------------------------------
template <typename TC, int Pts>
__device__ __forceinline__ void l2g_rows_lds(const unsigned char *lds, int capc, int o, int e0, const TC *wxc,
                                             const double *wy, double ly[5]) {
#pragma unroll
  for (int b = 0; b < Pts; b++) {
    TC p5[5] = {0, 0, 0, 0, 0};
    if constexpr (sizeof(TC) == 4) {
      const float4 *r4 = (const float4 *)lds + o + b * e0;
      const float *r1 = (const float *)(lds + 16 * capc) + o + b * e0;
      float4 w4[Pts];
      float w1[Pts];
#pragma unroll
      for (int a = 0; a < Pts; a++) {
        w4[a] = r4[a];
        w1[a] = r1[a];
      }
#pragma unroll
      for (int a = 0; a < Pts; a++) {
        p5[0] = fmaf(wxc[a], w4[a].x, p5[0]);
        p5[1] = fmaf(wxc[a], w4[a].y, p5[1]);
        p5[2] = fmaf(wxc[a], w4[a].z, p5[2]);
        p5[3] = fmaf(wxc[a], w4[a].w, p5[3]);
        p5[4] = fmaf(wxc[a], w1[a], p5[4]);
      }
    } else {
      const double2 *ra = (const double2 *)lds + o + b * e0;
      const double2 *rb = (const double2 *)(lds + 16 * capc) + o + b * e0;
      const double *rc = (const double *)(lds + 32 * capc) + o + b * e0;
#pragma unroll
      for (int a = 0; a < Pts; a++) {
        const double2 x01 = ra[a], x23 = rb[a];
        p5[0] = fma(wxc[a], x01.x, p5[0]);
        p5[1] = fma(wxc[a], x01.y, p5[1]);
        p5[2] = fma(wxc[a], x23.x, p5[2]);
        p5[3] = fma(wxc[a], x23.y, p5[3]);
        p5[4] = fma(wxc[a], rc[a], p5[4]);
      }
    }
#pragma unroll
    for (int f = 0; f < 5; f++) ly[f] = fma(wy[b], (double)p5[f], ly[f]);
  }
}

// A point's stencil straight from global memory (rare: an item whose donor box
// does not fit the LDS tile).  The thread's z-layers (g and g + 3, or g alone
// for K = 6), each summed as in l2g_rows_lds and combined as in the staged
// path, in loops that are not unrolled (the weights picked by selects).  The
// point is located and weighted again here with the same functions as the
// kernel's setup, so only scalars cross the call: an array argument of a
// function that is not inlined lives in scratch memory, and the kernel would
// store its weights there for every item, whichever path the item takes.
struct Sum5 {
  double v[5];
};

template <typename TB, typename TC, int Pts>
__device__ __noinline__ Sum5 l2g_point_global(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose,
                                              int d, int i, int j, int k, int sv, int stage, int g, int K) {
  const PatchDev &G0 = P[0];
  const PatchDev &D = P[d];
  const double X[3] = {xnum(G0, 0, i), xnum(G0, 1, j), xnum(G0, 2, k)};
  double xd[3], q[3];
  inv_map(D, pose[d], X, xd);
  for (int a = 0; a < 3; a++) q[a] = (xd[a] - D.lo[a]) * D.idx[a] - 0.5;
  double wx[Pts], wy[Pts], wz[Pts];
  const int s0 = lagrange_wt<Pts>(q[0], wx);
  const int s1 = lagrange_wt<Pts>(q[1], wy);
  const int s2 = lagrange_wt<Pts>(q[2], wz);
  TC wxc[Pts];
#pragma unroll
  for (int m = 0; m < Pts; m++) wxc[m] = (TC)wx[m];
  const TB *T = stage_buf<TB>(D, sv, stage);
  const uint32_t fs = (uint32_t)D.fstride;
  Sum5 part = {{0, 0, 0, 0, 0}};
  for (int m = 0; m < 2; m++) {
    const int cc = g + 3 * m;
    if (cc >= Pts || (K == 6 && m > 0)) break;
    int kk = s2 + cc;
    if (D.periodic[2]) kk = ((kk % D.n[2]) + D.n[2]) % D.n[2];
    double ly[5] = {0, 0, 0, 0, 0};
    for (int b = 0; b < Pts; b++) {
      int jj = s1 + b;
      if (D.periodic[1]) jj = ((jj % D.n[1]) + D.n[1]) % D.n[1];
      TC p5[5] = {0, 0, 0, 0, 0};
      for (int a = 0; a < Pts; a++) {
        int ii = s0 + a;
        if (D.periodic[0]) ii = ((ii % D.n[0]) + D.n[0]) % D.n[0];
        const uint32_t x = (uint32_t)cell_index(D, ii, jj, kk);
        TC w = (TC)0;
#pragma unroll
        for (int e = 0; e < Pts; e++) w = (e == a) ? wxc[e] : w;
#pragma unroll
        for (int f = 0; f < 5; f++) {
          const TC u = (TC)gld(T, f * fs + x);
          if constexpr (sizeof(TC) == 4) p5[f] = fmaf(w, u, p5[f]);
          else p5[f] = fma(w, u, p5[f]);
        }
      }
      double wb = 0.0;
#pragma unroll
      for (int e = 0; e < Pts; e++) wb = (e == b) ? wy[e] : wb;
#pragma unroll
      for (int f = 0; f < 5; f++) ly[f] = fma(wb, (double)p5[f], ly[f]);
    }
    double wzc = 0.0;
#pragma unroll
    for (int e = 0; e < Pts; e++) wzc = (e == cc) ? wz[e] : wzc;
#pragma unroll
    for (int f = 0; f < 5; f++) part.v[f] = __dadd_rn(part.v[f], __dmul_rn(wzc, ly[f]));
  }
  return part;
}

template <typename TB, typename TC, int Pts>
__global__ __launch_bounds__(L2G_THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_l2g_bucket(
    const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, const int32_t *list, const int2 *items,
    const int *nitems, int run, const int32_t *cover, int sv, int stage, unsigned long long *skips, FallbackRec *fb,
    int *fb_count, int force_direct) {
  constexpr int NW = L2G_THREADS / 64;
  constexpr int CAPC = L2G_LDS_BYTES / (5 * sizeof(TC));  // box cells: five fields a cell
  static_assert(L2G_ITEM * 3 <= L2G_THREADS && L2G_ITEM <= 64, "three threads per point of an item");
  static_assert(5 * L2G_THREADS * sizeof(double) <= L2G_LDS_BYTES, "partial sums fit the box LDS");
  __shared__ __align__(16) unsigned char lds_box[L2G_LDS_BYTES];
  __shared__ int wbox[NW][8];  // per wavefront: lowest / highest donor index per axis, donor patch range
  double(*red)[L2G_THREADS] = (double(*)[L2G_THREADS])lds_box;  // partial sums, once the box is done
  const PatchDev &G0 = P[0];
  if (!(G0.sv_mask & (1u << sv))) return;
  TB *TG = stage_buf<TB>(G0, sv, stage);
  const int tid = threadIdx.x;
  const int ni = nitems[0];
  const int nv = (ni + 8 * run - 1) / (8 * run) * (8 * run);
  for (int vb = blockIdx.x; vb < nv; vb += gridDim.x) {
    // runs of `run` consecutive items (neighbouring donor buckets) on one XCD
    const int item = xcd_spread(vb, run);
    if (item >= ni) continue;
    const int2 it = items[item];
    const int npts = it.y;
    const int K = npts <= L2G_THREADS / 6 ? 6 : 3;
    const bool act = tid < K * npts;
    const int pi = act ? tid % npts : 0, g = act ? tid / npts : 0;
    const long long c = act ? list[it.x + pi] : 0;
    const int i = (int)(c % G0.n[0]), j = (int)((c / G0.n[0]) % G0.n[1]),
              k = (int)(c / ((long long)G0.n[0] * G0.n[1]));
    const int d = act ? cover[c] : 0;
    bool valid = act && d >= 1 && (P[d].sv_mask & (1u << sv));
    int s[3] = {0, 0, 0};
    double xd[3] = {0, 0, 0};
    TC wxc[Pts];
    double wy[Pts], wz[Pts];
#pragma unroll
    for (int m = 0; m < Pts; m++) { wxc[m] = (TC)0; wy[m] = 0.0; wz[m] = 0.0; }
    if (valid) {
      const PatchDev &D = P[d];
      const double X[3] = {xnum(G0, 0, i), xnum(G0, 1, j), xnum(G0, 2, k)};
      inv_map(D, pose[d], X, xd);
      double q[3];
      for (int a = 0; a < 3; a++) {
        q[a] = (xd[a] - D.lo[a]) * D.idx[a] - 0.5;
        valid = valid && (q[a] > -1.0e6 && q[a] < 1.0e6);
      }
      if (valid) {
        double wx[Pts];
        s[0] = lagrange_wt<Pts>(q[0], wx);
        s[1] = lagrange_wt<Pts>(q[1], wy);
        s[2] = lagrange_wt<Pts>(q[2], wz);
#pragma unroll
        for (int m = 0; m < Pts; m++) wxc[m] = (TC)wx[m];
        for (int a = 0; a < 3; a++)
          if (!D.periodic[a] && (s[a] < 0 || s[a] + Pts - 1 > D.n[a] - 1)) valid = false;
      }
    }
    // the item's donor box and donor patch: reduced within each wavefront by
    // xor shuffles, the wavefronts' results combined through LDS
    {
      int v8[8];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        v8[a] = valid ? s[a] : (1 << 30);
        v8[3 + a] = valid ? s[a] + Pts - 1 : -(1 << 30);
      }
      v8[6] = valid ? d : (1 << 30);
      v8[7] = valid ? d : -1;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; a++) v8[a] = min(v8[a], __shfl_xor(v8[a], off));
#pragma unroll
        for (int a = 3; a < 6; a++) v8[a] = max(v8[a], __shfl_xor(v8[a], off));
        v8[6] = min(v8[6], __shfl_xor(v8[6], off));
        v8[7] = max(v8[7], __shfl_xor(v8[7], off));
      }
      if ((tid & 63) == 0)
#pragma unroll
        for (int a = 0; a < 8; a++) wbox[tid >> 6][a] = v8[a];
    }
    __syncthreads();
    int lo[3], hi[3], dmin, dmax;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      lo[a] = wbox[0][a];
      hi[a] = wbox[0][3 + a];
    }
    dmin = wbox[0][6];
    dmax = wbox[0][7];
#pragma unroll
    for (int w = 1; w < NW; w++) {
#pragma unroll
      for (int a = 0; a < 3; a++) {
        lo[a] = min(lo[a], wbox[w][a]);
        hi[a] = max(hi[a], wbox[w][3 + a]);
      }
      dmin = min(dmin, wbox[w][6]);
      dmax = max(dmax, wbox[w][7]);
    }
    const int e0 = hi[0] - lo[0] + 1, e1 = hi[1] - lo[1] + 1, e2 = hi[2] - lo[2] + 1;
    const int e01 = e0 * e1;
    const bool boxed = !force_direct && dmax >= 1 && dmin == dmax && e01 <= CAPC;
    // this thread's layers g, g + K of its point, summed into part in the
    // fixed grouping (each layer sum rounded on its own before the add)
    double part[5] = {0, 0, 0, 0, 0};
    double wzl[2] = {0.0, 0.0};  // z weights of the thread's two layers
#pragma unroll
    for (int m = 0; m < Pts; m++) {
      wzl[0] = (m == g) ? wz[m] : wzl[0];
      wzl[1] = (m == g + 3) ? wz[m] : wzl[1];
    }
    if (boxed) {
      const PatchDev &D = P[dmin];  // uniform: scalar loads
      const TB *T = stage_buf<TB>(D, sv, stage);
      const uint32_t fs = (uint32_t)D.fstride, dsy = (uint32_t)D.pitch, dsz = (uint32_t)D.slab;
      const int dn0 = D.n[0], dn1 = D.n[1], dn2 = D.n[2];
      const bool per0 = D.periodic[0] != 0, per1 = D.periodic[1] != 0, per2 = D.periodic[2] != 0;
      const int nzc = CAPC / e01;
      // flat box index q -> (x, row), row -> (b, layer) with float reciprocals:
      // exact, since (q + 0.5) / e lies at least 1/(2e) from an integer and q < 2^14
      const float ie0 = 1.0f / (float)e0, ie1 = 1.0f / (float)e1;
      for (int z0 = 0; z0 < e2; z0 += nzc) {
        const int nz = e2 - z0 < nzc ? e2 - z0 : nzc;
        const int v = e01 * nz;
        for (int q0 = tid; q0 < v; q0 += 4 * L2G_THREADS) {
          TC tmp[4][5];
#pragma unroll
          for (int m = 0; m < 4; m++) {
            const int q = q0 + m * L2G_THREADS;
            if (q < v) {
              const int row = (int)(((float)q + 0.5f) * ie0);
              const int x = q - row * e0;
              const int cc = (int)(((float)row + 0.5f) * ie1);
              const int b = row - cc * e1;
              // box cells lie inside [0, n) on every axis once periodic axes wrap
              int ii = lo[0] + x, jj = lo[1] + b, kk = lo[2] + z0 + cc;
              if (per0) ii = ((ii % dn0) + dn0) % dn0;
              if (per1) jj = ((jj % dn1) + dn1) % dn1;
              if (per2) kk = ((kk % dn2) + dn2) % dn2;
              const uint32_t gi = (uint32_t)(ii + PW_OX) + (uint32_t)(jj + PW_NG) * dsy + (uint32_t)(kk + PW_NG) * dsz;
#pragma unroll
              for (int f = 0; f < 5; f++) tmp[m][f] = (TC)gld(T, (uint32_t)f * fs + gi);
            }
          }
#pragma unroll
          for (int m = 0; m < 4; m++) {
            const int q = q0 + m * L2G_THREADS;
            if (q < v) {
              if constexpr (sizeof(TC) == 4) {
                ((float4 *)lds_box)[q] = make_float4(tmp[m][0], tmp[m][1], tmp[m][2], tmp[m][3]);
                ((float *)(lds_box + 16 * CAPC))[q] = tmp[m][4];
              } else {
                ((double2 *)lds_box)[q] = make_double2(tmp[m][0], tmp[m][1]);
                ((double2 *)(lds_box + 16 * CAPC))[q] = make_double2(tmp[m][2], tmp[m][3]);
                ((double *)(lds_box + 32 * CAPC))[q] = tmp[m][4];
              }
            }
          }
        }
        __syncthreads();
        if (valid) {
          const int first = (s[1] - lo[1]) * e0 + (s[0] - lo[0]);
#pragma unroll
          for (int m = 0; m < 2; m++) {
            const int cc = g + 3 * m;
            if (cc >= Pts || (K == 6 && m > 0)) break;
            const int lz = s[2] - lo[2] + cc - z0;
            if (lz < 0 || lz >= nz) continue;
            double ly[5] = {0, 0, 0, 0, 0};
            l2g_rows_lds<TC, Pts>(lds_box, CAPC, lz * e01 + first, e0, wxc, wy, ly);
#pragma unroll
            for (int f = 0; f < 5; f++) part[f] = __dadd_rn(part[f], __dmul_rn(wzl[m], ly[f]));
          }
        }
        __syncthreads();
      }
    } else if (valid) {
      // (rare) the stencil straight from global memory, same arithmetic
      const Sum5 r = l2g_point_global<TB, TC, Pts>(P, pose, d, i, j, k, sv, stage, g, K);
#pragma unroll
      for (int f = 0; f < 5; f++) part[f] = r.v[f];
    }
    // the partial sums of a point's threads meet in its g = 0 thread (in the
    // box's LDS, which every thread is done with)
    __syncthreads();
    if (act && g > 0) {
#pragma unroll
      for (int f = 0; f < 5; f++) red[f][tid] = part[f];
    }
    __syncthreads();
    if (act && g == 0) {
      if (valid) {
        double acc[5];
        if (K == 3) {
#pragma unroll
          for (int f = 0; f < 5; f++)
            acc[f] = __dadd_rn(__dadd_rn(part[f], red[f][tid + npts]), red[f][tid + 2 * npts]);
        } else {
#pragma unroll
          for (int f = 0; f < 5; f++) {
            const double p0 = __dadd_rn(part[f], red[f][tid + 3 * npts]);
            const double p1 = __dadd_rn(red[f][tid + npts], red[f][tid + 4 * npts]);
            const double p2 = __dadd_rn(red[f][tid + 2 * npts], red[f][tid + 5 * npts]);
            acc[f] = __dadd_rn(__dadd_rn(p0, p1), p2);
          }
        }
        const PatchDev &D = P[d];
        double in4[4] = {acc[1], acc[2], acc[3], acc[4]}, G[3], pit, out[5];
        const double X[3] = {xnum(G0, 0, i), xnum(G0, 1, j), xnum(G0, 2, k)};
        patch_to_bg_at(D, pose[d], X, xd, in4, pit, G);
        // the global patch's numerical frame is the background frame
        out[0] = acc[0];
        out[1] = pit;
        for (int m = 0; m < 3; m++) out[2 + m] = G[m];
        const long long dst = cell_index(G0, i, j, k);
        for (int f = 0; f < 5; f++) TG[f * G0.fstride + dst] = (TB)out[f];
      } else {
        atomicAdd(skips, 1ull);
        const int slot = atomicAdd(fb_count, 1);
        fb[slot] = FallbackRec{0, 1, (uint32_t)c};
      }
    }
    __syncthreads();
  }
}

// Work items of the local -> global kernel: every non-empty donor bucket cut
// into runs of at most L2G_ITEM consecutive entries of the sorted list
// (x: first entry, y: count).  The order of the items follows the atomics, the
// values they give do not depend on it.
__global__ void k_l2g_items(const int *cnt, const int *off, int nb, int2 *items, int *nitems) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int m = b < nb ? cnt[b] : 0;
  const int nch = (m + L2G_ITEM - 1) / L2G_ITEM;
  // the wavefront reserves its slots with one atomic (inclusive scan by shuffles)
  int incl = nch;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  int base = 0;
  if (lane == 63 && incl > 0) base = atomicAdd(nitems, incl);
  base = __shfl(base, 63);
  const int slot = base + incl - nch;
  for (int q = 0; q < nch; q++) items[slot + q] = make_int2(off[b] + q * L2G_ITEM, min(L2G_ITEM, m - q * L2G_ITEM));
}

// Local ghost cells of a state vector that the global patch does not carry
// have no donor: they keep their lower-priority value, the registered exact
// solution, written here directly (one thread per ghost cell of the brick
// list) instead of through a fallback record per point.
template <typename TB>
__global__ __launch_bounds__(BRICK_THREADS) void k_g2l_exact(const PatchDev *__restrict__ P,
                                                           const PoseDev *__restrict__ pose, const GBrick *bricks,
                                                           int nbricks, int sv, int stage, const ExactDev *ex,
                                                           double v, const double *tdev, double tmul, double dt) {
  if ((int)blockIdx.x >= nbricks) return;
  const GBrick B = bricks[blockIdx.x];
  const PatchDev &r = P[B.patch];
  const int tid = threadIdx.x;
  if (tid >= B.di * B.dj * B.dk || !(r.sv_mask & (1u << sv))) return;
  const int c[3] = {B.i0 + tid % B.di, B.j0 + (tid / B.di) % B.dj, B.k0 + tid / (B.di * B.dj)};
  bool inside = true, winside = true;
  for (int a = 0; a < 3; a++) {
    inside = inside && c[a] >= 0 && c[a] < r.n[a];
    const int w = r.periodic[a] ? ((c[a] % r.n[a]) + r.n[a]) % r.n[a] : c[a];
    winside = winside && w >= 0 && w < r.n[a];
  }
  if (inside || winside) return;
  const double xr[3] = {xnum(r, 0, c[0]), xnum(r, 1, c[1]), xnum(r, 2, c[2])};
  double out[5];
  exact_patch(ex[sv], v, r, pose[B.patch], tdev[0] + tmul * dt, xr, out);
  TB *TR = stage_buf<TB>(r, sv, stage);
  const long long dst = cell_index(r, c[0], c[1], c[2]);
  for (int f = 0; f < 5; f++) TR[f * r.fstride + dst] = (TB)out[f];
}

// Points that could not be interpolated keep their lower-priority value: a
// local ghost gets the exact solution (if registered) or a copy of the nearest
// interior cell; a global effective ghost gets the exact solution or NaN.
template <typename TB>
__global__ void k_fallback(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, const FallbackRec *fb, const int *fb_count, int sv,
                           int stage, const ExactDev *ex, double v, const double *tdev, double tmul, double dt) {
  const int n = fb_count[0];
  const double t = tdev[0] + tmul * dt;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const FallbackRec F = fb[q];
    const PatchDev &r = P[F.patch];
    int c[3];
    if (F.kind == 0) {
      c[0] = (int)(F.cell & 1023u) - PW_NG;
      c[1] = (int)((F.cell >> 10) & 1023u) - PW_NG;
      c[2] = (int)((F.cell >> 20) & 1023u) - PW_NG;
    } else {
      c[0] = (int)(F.cell % r.n[0]);
      c[1] = (int)((F.cell / r.n[0]) % r.n[1]);
      c[2] = (int)(F.cell / ((unsigned)r.n[0] * r.n[1]));
    }
    double xr[3] = {xnum(r, 0, c[0]), xnum(r, 1, c[1]), xnum(r, 2, c[2])}, out[5];
    TB *TR = stage_buf<TB>(r, sv, stage);
    if (ex[sv].kind != EX_NONE) {
      exact_patch(ex[sv], v, r, pose[F.patch], t, xr, out);
    } else if (F.kind == 0) {
      int w[3];
      for (int a = 0; a < 3; a++) {
        w[a] = c[a];
        if (r.periodic[a]) w[a] = ((c[a] % r.n[a]) + r.n[a]) % r.n[a];
        w[a] = w[a] < 0 ? 0 : (w[a] >= r.n[a] ? r.n[a] - 1 : w[a]);
      }
      const long long src = cell_index(r, w[0], w[1], w[2]);
      for (int f = 0; f < 5; f++) out[f] = (double)TR[f * r.fstride + src];
    } else {
      for (int f = 0; f < 5; f++) out[f] = NAN;
    }
    const long long dst = cell_index(r, c[0], c[1], c[2]);
    for (int f = 0; f < 5; f++) TR[f * r.fstride + dst] = (TB)out[f];
  }
}

// End of step: cells live now but not live during the step get u_{n+1}
// interpolated from the covering local patch; cells that become deactivated are
// poisoned (nothing writes a deactivated cell, so it stays poisoned); the new
// flags become current.  mode 0: first flags (no uncover fill, every deactivated
// cell poisoned).  Two kernels: k_finalize streams the flags and cover ids
// (sixteen cells per thread, 16-byte words), poisons in place and lists the
// cells that become live; k_uncover fills the listed cells.
__device__ inline void poison_cell(const PatchDev &G0, long long c, int nsv) {
  const int i = (int)(c % G0.n[0]), j = (int)((c / G0.n[0]) % G0.n[1]),
            k = (int)(c / ((long long)G0.n[0] * G0.n[1]));
  const long long x = cell_index(G0, i, j, k);
  for (int sv = 0; sv < nsv; sv++) {
    if (!(G0.sv_mask & (1u << sv))) continue;
    for (int f = 0; f < 5; f++) G0.u[sv][f * G0.fstride + x] = NAN;
    if (G0.us[sv])
      for (int f = 0; f < 5; f++) G0.us[sv][f * G0.fstride + x] = NAN;
  }
}

#define FIN_CELLS 16
__global__ __launch_bounds__(256) void k_finalize(const PatchDev *__restrict__ P, uint8_t *flag_cur,
                                                  const uint8_t *flag_new, int32_t *cover_cur, int32_t *cover_new,
                                                  int nsv, int mode, int2 *ulist, int *ucount) {
  const PatchDev &G0 = P[0];
  const long long total = (long long)G0.n[0] * G0.n[1] * G0.n[2];
  const long long c0 = (long long)FIN_CELLS * ((long long)blockIdx.x * blockDim.x + threadIdx.x);
  if (c0 >= total) return;
  if (c0 + FIN_CELLS <= total) {
    const uint4 fo16 = *(const uint4 *)(flag_cur + c0), fn16 = *(const uint4 *)(flag_new + c0);
    const uint32_t fow[4] = {fo16.x, fo16.y, fo16.z, fo16.w}, fnw[4] = {fn16.x, fn16.y, fn16.z, fn16.w};
    uint32_t up = 0, pz = 0;  // cells to fill (become live) and to poison (become deactivated)
#pragma unroll
    for (int m = 0; m < FIN_CELLS; m++) {
      const uint8_t fo = (uint8_t)(fow[m >> 2] >> (8 * (m & 3))), fn = (uint8_t)(fnw[m >> 2] >> (8 * (m & 3)));
      up |= (uint32_t)(mode == 1 && fo != LIVE && fn == LIVE) << m;
      pz |= (uint32_t)(fn == DEACT && (mode == 0 || fo != DEACT)) << m;
    }
    while (up) {
      const int m = __ffs(up) - 1;
      up &= up - 1;
      ulist[atomicAdd(ucount, 1)] = make_int2((int)(c0 + m), cover_cur[c0 + m]);
    }
    while (pz) {
      const int m = __ffs(pz) - 1;
      pz &= pz - 1;
      poison_cell(G0, c0 + m, nsv);
    }
#pragma unroll
    for (int w = 0; w < 4; w++) {
      *(int4 *)(cover_cur + c0 + 4 * w) = *(const int4 *)(cover_new + c0 + 4 * w);
      *(int4 *)(cover_new + c0 + 4 * w) = make_int4(-1, -1, -1, -1);
    }
    *(uint4 *)(flag_cur + c0) = fn16;
  } else {
    for (long long c = c0; c < total; c++) {
      const uint8_t fo = flag_cur[c], fn = flag_new[c];
      if (mode == 1 && fo != LIVE && fn == LIVE) ulist[atomicAdd(ucount, 1)] = make_int2((int)c, cover_cur[c]);
      if (fn == DEACT && (mode == 0 || fo != DEACT)) poison_cell(G0, c, nsv);
      flag_cur[c] = fn;
      cover_cur[c] = cover_new[c];
      cover_new[c] = -1;
    }
  }
}

// Weight of node m of the P-point Lagrange stencil at position t from its first
// node (the same product as lagrange_w).
__device__ inline double lagrange_node(int P, double t, int m) {
  double num = 1.0, den = 1.0;
  for (int l = 0; l < P; l++) {
    if (l == m) continue;
    num *= (t - (double)l);
    den *= (double)(m - l);
  }
  return num / den;
}

// The uncover fill of the listed cells (after k_finalize: cover_cur holds the
// new cover ids).  The donor is the patch covering the cell now, else the one
// that covered it during the step.  One wavefront per cell: every lane locates
// the point (FP64), lane (a, b) < P^2 sums x-node a of row b over the z-layers
// of the stencil, and the five partial sums are reduced across the wavefront.
__global__ __launch_bounds__(256) void k_uncover(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose,
                                                 const int2 *ulist, const int *ucount, const int32_t *cover_cur,
                                                 int nsv, const int *Pts, const ExactDev *ex, const double *vs,
                                                 const double *tdev, unsigned long long *counters) {
  const PatchDev &G0 = P[0];
  const int n = ucount[0];
  const int lane = threadIdx.x & 63;
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  for (int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < n; q += nwaves) {
    const long long c = ulist[q].x;
    const int co = ulist[q].y, cn = cover_cur[c];
    const int i = (int)(c % G0.n[0]), j = (int)((c / G0.n[0]) % G0.n[1]),
              k = (int)(c / ((long long)G0.n[0] * G0.n[1]));
    const long long x = cell_index(G0, i, j, k);
    const int d = cn >= 1 ? cn : co;
    const PatchDev &D = P[d >= 1 ? d : 0];
    const double xr[3] = {xnum(G0, 0, i), xnum(G0, 1, j), xnum(G0, 2, k)};
    double X[3], xd[3];
    global_X(G0, pose[0], i, j, k, X);
    if (d >= 1) inv_map(D, pose[d], X, xd);
    if (lane == 0) atomicAdd(&counters[3], 1ull);
    for (int sv = 0; sv < nsv; sv++) {
      if (!(G0.sv_mask & (1u << sv))) continue;
      const int Pn = Pts[sv];
      bool ok = d >= 1 && (D.sv_mask & (1u << sv));
      int s[3] = {0, 0, 0};
      double t[3] = {0, 0, 0};
      for (int a = 0; a < 3 && ok; a++) {
        const double qa = (xd[a] - D.lo[a]) * D.idx[a] - 0.5;
        ok = qa > -1.0e6 && qa < 1.0e6;
        if (!ok) break;
        s[a] = (int)floor(qa - 0.5 * (Pn - 2));
        t[a] = qa - (double)s[a];
        ok = D.periodic[a] || (s[a] >= 0 && s[a] + Pn - 1 <= D.n[a] - 1);
      }
      double out[5];
      if (ok) {
        double acc[5] = {0, 0, 0, 0, 0};
        if (lane < Pn * Pn) {
          const int a = lane % Pn, b = lane / Pn;
          int ii = s[0] + a, jj = s[1] + b;
          if (D.periodic[0]) ii = ((ii % D.n[0]) + D.n[0]) % D.n[0];
          if (D.periodic[1]) jj = ((jj % D.n[1]) + D.n[1]) % D.n[1];
          const double wxy = lagrange_node(Pn, t[0], a) * lagrange_node(Pn, t[1], b);
          const double *U = D.u[sv];
          for (int cz = 0; cz < Pn; cz++) {
            int kk = s[2] + cz;
            if (D.periodic[2]) kk = ((kk % D.n[2]) + D.n[2]) % D.n[2];
            const long long xs = cell_index(D, ii, jj, kk);
            const double w = wxy * lagrange_node(Pn, t[2], cz);
            for (int f = 0; f < 5; f++) acc[f] += w * U[f * D.fstride + xs];
          }
        }
        for (int f = 0; f < 5; f++)
          for (int m = 32; m >= 1; m >>= 1) acc[f] += __shfl_xor(acc[f], m);
        double in4[4] = {acc[1], acc[2], acc[3], acc[4]}, G[3], pit, o4[4];
        patch_to_bg_at(D, pose[d], X, xd, in4, pit, G);
        bg_to_patch(G0, pose[0], xr, pit, G, o4);
        out[0] = acc[0];
        for (int m = 0; m < 4; m++) out[1 + m] = o4[m];
      } else {
        if (lane == 0) atomicAdd(&counters[2], 1ull);
        if (ex[sv].kind != EX_NONE) exact_patch(ex[sv], vs[sv], G0, pose[0], tdev[0], xr, out);
        else for (int f = 0; f < 5; f++) out[f] = NAN;
      }
      if (lane == 0) {
        for (int f = 0; f < 5; f++) G0.u[sv][f * G0.fstride + x] = out[f];
        if (G0.us[sv])
          for (int f = 0; f < 5; f++) G0.us[sv][f * G0.fstride + x] = (float)out[f];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// RHS of Eqs. eom1-eom3 (source S = 0) with Kreiss-Oliger dissipation on all
// five fields, fused with the classic-RK4 stage update.
//
// Metric terms (flat background with wave speed v, patch map X = c(t) + R(t) M(x')):
//   b = R^T c', a = R^T c'' (patch axes), beta = K b with K = (dM/dx')^-1,
//   dPi_t/dt = m.D phi + 2 beta.D Pi_t + sum_i (v^2 h_i - beta_i^2) D_ii phi
//              - 2 sum_{i<j} beta_i beta_j D_ij phi
// Cartesian: h = 1, m = a.  Spherical: h = (1, 1/r^2, 1/(r sin th)^2) and
//   m = K a - Q(b) + v^2 (2/r, cot th / r^2, 0), Q the coordinate acceleration of
//   straight-line motion in spherical coordinates.  Cylindrical (r, phi, z):
//   h = (1, 1/r^2, 1), Q(b) = (b_phi^2 / r, -2 b_r b_phi / r^2, 0) with b_r, b_phi
//   the components along e_r, e_phi, and m = K a - Q(b) + v^2 (1/r, 0, 0).
// A patch rotating with angular velocity w (wp = R^T w) has, at y = M(x'), the
// position-dependent b + wp x y in place of b and a - 2 wp x b - wp x (wp x y)
// in place of a (frame_terms).
// FORM = 1 is the first-order reduction of the same equation: the evolved
// Psi_i = Pi_i stands for D_i phi and D_i Psi_j for D_ij phi (the off-diagonal
// pairs as (D_i Psi_j + D_j Psi_i) / 2), so no second differences of phi enter.
//
// Tiling (2.5-D): a workgroup owns a 32 x 8 column tile and marches through the
// tile's planes in z (a tuning parameter).  Each thread keeps its column's
// 7-plane window of the 5 fields in registers (z stencils) and a 5-plane window
// of D_x phi, D_y phi (mixed x-z and y-z derivatives as D_z of D_x phi, D_y phi).
// The centre plane of the 5 fields and the phi plane one below the newest are
// staged in LDS with a 3-cell x-y halo for the x-y stencils.
// ---------------------------------------------------------------------------
template <typename TIN, typename TOUT, typename TC, int STAGE, int COORD, bool GLOB, int AM, int FORM, int SH>
__global__ __launch_bounds__((StageTile<GLOB, SH>::THREADS)) void k_stage(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose_slot, const TileRec *tiles,
                                               int ntiles, int chunk, const uint8_t *gflag, int sv, double dt,
                                               double v2, double eps) {
  using TL = StageTile<GLOB, SH>;
  constexpr int ST_TX = TL::TX, ST_TY = TL::TY, ST_PX = TL::PX, ST_PW = TL::PW;
  constexpr int ST_THREADS = TL::THREADS;
  __shared__ TC Bc[2][5][ST_PW];
  __shared__ TC Ad[2][ST_PW];
  const int bid = blockIdx.x;
  const int tidx = (bid & 7) * chunk + (bid >> 3);  // contiguous tile runs per XCD
  if (tidx >= ntiles) return;
  const TileRec tl = tiles[tidx];
  const PatchDev &p = P[tl.patch];
  const PoseDev &ps = pose_slot[tl.patch];
  const int tid = threadIdx.x;
  // a thread owns column tx of RY tile rows: ty, ty + TYH, ...
  constexpr int RY = TL::RY, TYH = ST_TY / RY;
  const int tx = tid % ST_TX, ty = tid / ST_TX;
  const int i = tl.x0 + tx;
  int jr[RY], ownr[RY];
  bool inpadr[RY], icolr[RY];
  uint32_t colr[RY];
  const int z0 = tl.z0;
  const int nz = tl.nz;
  const TIN *in = (const TIN *)(STAGE == 0 ? (sizeof(TIN) == 8 ? (const void *)p.u[sv] : (const void *)p.us[sv])
                                            : (STAGE == 2 ? p.vb[sv] : p.va[sv]));
  float *Us = p.us[sv];  // FP32 copy of u (mixed path): written with u_{n+1} by the last stage
  TOUT *vout = (TOUT *)(STAGE == 1 ? p.vb[sv] : p.va[sv]);
  double *U = p.u[sv];
  double *Acc = p.acc[sv];
  // mixed path (FP32 stage values): stages 2-3 build v_{s+1} on the FP32 copy of
  // u_n; the accumulator is FP64 u_n + dt sum_l b_l K_l (AM = 0) or the FP32
  // increment dt sum_l b_l K_l (AM = 1)
  constexpr bool MIX = sizeof(TOUT) == 4;
  constexpr bool INC = MIX && AM == 1;
  float *AccF = (float *)p.acc[sv];
  // 32-bit element offsets: the host keeps the five fields of a patch (5 fstride
  // elements, ghosts and row padding included) below 2^32 elements
  const uint32_t fs = (uint32_t)p.fstride, sz = (uint32_t)p.slab;
#pragma unroll
  for (int r = 0; r < RY; r++) {
    jr[r] = tl.y0 + ty + r * TYH;
    inpadr[r] = (i < p.n[0] + PW_NG) && (jr[r] < p.n[1] + PW_NG);
    icolr[r] = (i < p.n[0]) && (jr[r] < p.n[1]);
    colr[r] = (uint32_t)cell_index(p, i, jr[r], 0);
    ownr[r] = (ty + r * TYH + 3) * ST_PX + (tx + 3);
  }
  // halo cells of the LDS planes: the ring of ST_PW - ST_THREADS cells around
  // the tile, enumerated row by row; thread t takes ring cells t, t + ST_THREADS
  constexpr int NHALO = ST_PW - ST_TX * ST_TY;
  constexpr int NH = (NHALO + ST_THREADS - 1) / ST_THREADS;
  uint32_t hoff[NH];
  bool hval[NH];
  int hslot[NH];
#pragma unroll
  for (int m = 0; m < NH; m++) {
    const int h = tid + ST_THREADS * m;
    hval[m] = false;
    hoff[m] = 0;
    hslot[m] = 0;
    if (h < NHALO) {
      int hx, hy;
      if (h < 3 * ST_PX) {  // three rows below the tile
        hx = h % ST_PX;
        hy = h / ST_PX;
      } else if (h < 3 * ST_PX + 6 * ST_TY) {  // 3 + 3 side cells of the tile rows
        const int r = h - 3 * ST_PX;
        hy = 3 + r / 6;
        const int sx = r % 6;
        hx = sx < 3 ? sx : ST_TX + sx;
      } else {  // three rows above the tile
        const int r = h - 3 * ST_PX - 6 * ST_TY;
        hx = r % ST_PX;
        hy = 3 + ST_TY + r / ST_PX;
      }
      hslot[m] = hy * ST_PX + hx;
      const int gi = tl.x0 - 3 + hx, gj = tl.y0 - 3 + hy;
      if (gi < p.n[0] + PW_NG && gj < p.n[1] + PW_NG) {
        hval[m] = true;
        hoff[m] = (uint32_t)cell_index(p, gi, gj, 0);
      }
    }
  }
  const TC i12dx[3] = {(TC)(p.idx[0] / 12.0), (TC)(p.idx[1] / 12.0), (TC)(p.idx[2] / 12.0)};
  const TC i12dx2[3] = {(TC)(p.idx[0] * p.idx[0] / 12.0), (TC)(p.idx[1] * p.idx[1] / 12.0),
                        (TC)(p.idx[2] * p.idx[2] / 12.0)};
  const TC ko[3] = {(TC)(eps / 64.0 * p.idx[0]), (TC)(eps / 64.0 * p.idx[1]), (TC)(eps / 64.0 * p.idx[2])};
  // rotating patches: position-dependent shift and acceleration (frame_terms).
  // The global patch is the static background frame: no shift, no mixed
  // derivatives, so it needs no D_x phi, D_y phi window (DWIN)
  const bool spin = !GLOB && ((ps.wp[0] != 0.0) || (ps.wp[1] != 0.0) || (ps.wp[2] != 0.0));
  const bool moving = !GLOB && (spin || (ps.b[0] != 0.0) || (ps.b[1] != 0.0) || (ps.b[2] != 0.0));
  constexpr bool DWIN = FORM == 0 && !GLOB;
  static_assert(RY == 1 || !DWIN, "several rows per thread only without the D_x phi, D_y phi window");
  const double bdt = STAGE == 0 ? dt / 6.0 : (STAGE == 3 ? dt / 6.0 : dt / 3.0);
  const double adt = STAGE == 2 ? dt : dt / 2.0;
  const float bdtf = (float)bdt, adtf = (float)adt;
  TC qr[RY][5][7];
  TC dqx[5], dqy[5];
#pragma unroll
  for (int r = 0; r < RY; r++)
#pragma unroll
    for (int f = 0; f < 5; f++)
#pragma unroll
      for (int d = 0; d < 7; d++) qr[r][f][d] = (TC)0;
#pragma unroll
  for (int d = 0; d < 5; d++) { dqx[d] = (TC)0; dqy[d] = (TC)0; }
  const TC w1[5] = {(TC)1, (TC)-8, (TC)0, (TC)8, (TC)-1};

  // software pipeline: the loads of iteration it+1 are in flight while
  // iteration it computes
  TC pown[RY][5], phA[NH], phB[NH][5];
  auto prefetch = [&](int itp) {
    const int zn = z0 - 3 + itp;
    const uint32_t zo = (uint32_t)(zn + PW_NG) * sz;  // cell_index already holds the +NG of z = 0
#pragma unroll
    for (int r = 0; r < RY; r++)
#pragma unroll
      for (int f = 0; f < 5; f++) pown[r][f] = inpadr[r] ? (TC)gld(in, f * fs + colr[r] + zo - PW_NG * sz) : (TC)0;
    if (DWIN && itp >= 2) {
      const uint32_t za = zo - (PW_NG + 1) * sz;
#pragma unroll
      for (int m = 0; m < NH; m++) phA[m] = hval[m] ? (TC)gld(in, hoff[m] + za) : (TC)0;
    }
    if (itp >= 6) {
      const uint32_t zb = zo - (PW_NG + 3) * sz;
#pragma unroll
      for (int m = 0; m < NH; m++)
#pragma unroll
        for (int f = 0; f < 5; f++) phB[m][f] = hval[m] ? (TC)gld(in, f * fs + hoff[m] + zb) : (TC)0;
    }
  };
  // Warm-up, all at once instead of six serial plane steps: the own-column
  // values of planes z0-3 .. z0+2 go to the z-window, and D_x phi, D_y phi at
  // planes z0-2 .. z0+1 are formed from phi planes staged with their halo rings
  // (in the second centre-plane buffer, first written two iterations later).
  if (DWIN) {
    TC(&q)[5][7] = qr[0];  // RY == 1 with the window
    const int own = ownr[0];
    const bool inpad = inpadr[0], icol = icolr[0];
    const uint32_t col = colr[0];
    TC wh[4][NH];
#pragma unroll
    for (int w = 0; w < 6; w++) {
      const uint32_t zo = (uint32_t)(z0 - 3 + w + PW_NG) * sz - PW_NG * sz;
#pragma unroll
      for (int f = 0; f < 5; f++) q[f][w + 1] = inpad ? (TC)gld(in, f * fs + col + zo) : (TC)0;
    }
#pragma unroll
    for (int w = 0; w < 4; w++) {
      const uint32_t zo = (uint32_t)(z0 - 2 + w + PW_NG) * sz - PW_NG * sz;
#pragma unroll
      for (int m = 0; m < NH; m++) wh[w][m] = hval[m] ? (TC)gld(in, hoff[m] + zo) : (TC)0;
    }
    prefetch(6);
#pragma unroll
    for (int w = 0; w < 4; w++) {
      TC *A_ = Bc[1][w];
      if (inpad) A_[own] = q[0][w + 2];
#pragma unroll
      for (int m = 0; m < NH; m++)
        if (hval[m]) A_[hslot[m]] = wh[w][m];
    }
    __syncthreads();
    if (icol) {
#pragma unroll
      for (int w = 0; w < 4; w++) {
        const TC *A_ = Bc[1][w];
        dqx[w + 1] = ((A_[own - 2] - A_[own + 2]) + (TC)8 * (A_[own + 1] - A_[own - 1])) * i12dx[0];
        dqy[w + 1] =
            ((A_[own - 2 * ST_PX] - A_[own + 2 * ST_PX]) + (TC)8 * (A_[own + ST_PX] - A_[own - ST_PX])) * i12dx[1];
      }
    }
  } else {
    // first-order form or the static global patch: no D_x phi, D_y phi window;
    // the z-window and the prefetch only
#pragma unroll
    for (int w = 0; w < 6; w++) {
      const uint32_t zo = (uint32_t)(z0 - 3 + w + PW_NG) * sz - PW_NG * sz;
#pragma unroll
      for (int r = 0; r < RY; r++)
#pragma unroll
        for (int f = 0; f < 5; f++) qr[r][f][w + 1] = inpadr[r] ? (TC)gld(in, f * fs + colr[r] + zo) : (TC)0;
    }
    prefetch(6);
  }
  for (int it = 6; it < nz + 6; it++) {
    const int zn = z0 - 3 + it;
    const int buf = it & 1;
#pragma unroll
    for (int r = 0; r < RY; r++)
#pragma unroll
      for (int f = 0; f < 5; f++) {
#pragma unroll
        for (int d = 0; d < 6; d++) qr[r][f][d] = qr[r][f][d + 1];
        qr[r][f][6] = pown[r][f];
      }
    const bool do_d = DWIN && it >= 2;  // phi plane zd = zn - 1 for D_x phi, D_y phi
    const bool do_c = it >= 6;  // centre plane zc = zn - 3
    TC *A_ = Ad[buf];
    if (do_d) {
      if (inpadr[0]) A_[ownr[0]] = qr[0][0][5];  // RY == 1 with the window
#pragma unroll
      for (int m = 0; m < NH; m++)
        if (hval[m]) A_[hslot[m]] = phA[m];
    }
    // centre-cell data of the RK update, issued before the barrier.  FP64 path:
    // u_n (stages 1-3) and the accumulator (stages 2-4).  Mixed path, FP64
    // accumulator: u_n (stage 1), the FP32 copy of u_n (stages 2-3), the
    // accumulator (stages 2-4).  Mixed path, FP32 increments: the FP32 copy of
    // u_n (stages 2-3; stage 1 has it in the z-window), the increment (stages
    // 2-4), u_n itself in stage 4 only.
    double cur_[RY][5], car_[RY][5];
    float cusr_[RY][5], cdr_[RY][5];
#pragma unroll
    for (int r = 0; r < RY; r++)
      if (do_c && icolr[r]) {
        const uint32_t xc = colr[r] + (uint32_t)(zn - 3) * sz;
#pragma unroll
        for (int f = 0; f < 5; f++) {
          cusr_[r][f] = (MIX && (STAGE == 1 || STAGE == 2)) ? gld((const float *)Us, f * fs + xc) : 0.0f;
          if (INC) {
            cdr_[r][f] = STAGE != 0 ? gld((const float *)AccF, f * fs + xc) : 0.0f;
            cur_[r][f] = STAGE == 3 ? gld(U, f * fs + xc) : 0.0;
            car_[r][f] = 0.0;
          } else if (MIX) {
            cdr_[r][f] = 0.0f;
            cur_[r][f] = STAGE == 0 ? gld(U, f * fs + xc) : 0.0;
            car_[r][f] = STAGE != 0 ? gld(Acc, f * fs + xc) : 0.0;
          } else {
            cdr_[r][f] = 0.0f;
            cur_[r][f] = STAGE != 3 ? gld(U, f * fs + xc) : 0.0;
            car_[r][f] = STAGE != 0 ? gld(Acc, f * fs + xc) : 0.0;
          }
        }
      }
    if (do_c) {
#pragma unroll
      for (int r = 0; r < RY; r++)
        if (inpadr[r]) {
#pragma unroll
          for (int f = 0; f < 5; f++) Bc[buf][f][ownr[r]] = qr[r][f][3];
        }
#pragma unroll
      for (int m = 0; m < NH; m++)
        if (hval[m]) {
#pragma unroll
          for (int f = 0; f < 5; f++) Bc[buf][f][hslot[m]] = phB[m][f];
        }
    }
    __syncthreads();
    if (it + 1 < nz + 6) prefetch(it + 1);
    if (do_d && icolr[0]) {
      const int own = ownr[0];  // RY == 1 with the window
#pragma unroll
      for (int d = 0; d < 4; d++) { dqx[d] = dqx[d + 1]; dqy[d] = dqy[d + 1]; }
      dqx[4] = ((A_[own - 2] - A_[own + 2]) + (TC)8 * (A_[own + 1] - A_[own - 1])) * i12dx[0];
      dqy[4] = ((A_[own - 2 * ST_PX] - A_[own + 2 * ST_PX]) + (TC)8 * (A_[own + ST_PX] - A_[own - ST_PX])) * i12dx[1];
    }
#pragma unroll
    for (int r = 0; r < RY; r++) {
      // row r of the thread, under the names of the one-row form
      TC(&q)[5][7] = qr[r];
      const int own = ownr[r], j = jr[r];
      const bool icol = icolr[r];
      const uint32_t col = colr[r];
      const double(&cu)[5] = cur_[r];
      const double(&ca)[5] = car_[r];
      const float(&cus)[5] = cusr_[r];
      const float(&cd)[5] = cdr_[r];
      if (do_c && icol) {
        const int k = zn - 3;
        bool live = true;
        if (GLOB && gflag) live = gflag[((long long)k * p.n[1] + j) * p.n[0] + i] == LIVE;
        if (live) {
          TC m_[3], b2_[3], h_[3], bb_[3];
          if (COORD == CART) {
            double bv[3] = {ps.b[0], ps.b[1], ps.b[2]}, av[3] = {ps.a[0], ps.a[1], ps.a[2]};
            if (spin) {
              const double y[3] = {p.lo[0] + (i + 0.5) * p.dx[0], p.lo[1] + (j + 0.5) * p.dx[1],
                                   p.lo[2] + (k + 0.5) * p.dx[2]};
              frame_terms(ps, y, bv, av);
            }
#pragma unroll
            for (int a = 0; a < 3; a++) {
              m_[a] = (TC)av[a];
              b2_[a] = (TC)(2.0 * bv[a]);
              h_[a] = (TC)(v2 - bv[a] * bv[a]);
            }
            bb_[0] = (TC)(2.0 * bv[0] * bv[1]);
            bb_[1] = (TC)(2.0 * bv[0] * bv[2]);
            bb_[2] = (TC)(2.0 * bv[1] * bv[2]);
          } else if (COORD == SPH) {
            const double r = p.lo[0] + (i + 0.5) * p.dx[0];
            double st, ct, sp, cp;
            trig_axis(p, 0, p.n[1] + 2 * PW_NG, j, st, ct);
            trig_axis(p, 2 * (p.n[1] + 2 * PW_NG), p.n[2] + 2 * PW_NG, k, sp, cp);
            const double er[3] = {st * cp, st * sp, ct}, et[3] = {ct * cp, ct * sp, -st}, ep[2] = {-sp, cp};
            double bv[3] = {ps.b[0], ps.b[1], ps.b[2]}, av[3] = {ps.a[0], ps.a[1], ps.a[2]};
            if (spin) {
              const double y[3] = {r * er[0], r * er[1], r * er[2]};
              frame_terms(ps, y, bv, av);
            }
            double ir = 1.0 / r, irs = ir / st, cot = ct / st;
            double br = er[0] * bv[0] + er[1] * bv[1] + er[2] * bv[2];
            double bt = et[0] * bv[0] + et[1] * bv[1] + et[2] * bv[2];
            double bp = ep[0] * bv[0] + ep[1] * bv[1];
            double ar = er[0] * av[0] + er[1] * av[1] + er[2] * av[2];
            double at = et[0] * av[0] + et[1] * av[1] + et[2] * av[2];
            double ap = ep[0] * av[0] + ep[1] * av[1];
            double beta[3] = {br, bt * ir, bp * irs};
            double Q0 = (bt * bt + bp * bp) * ir;
            double Q1 = (-2.0 * br * bt + bp * bp * cot) * ir * ir;
            double Q2 = -2.0 * bp * (br + bt * cot) * ir * irs;
            double mm[3] = {ar - Q0 + v2 * 2.0 * ir, at * ir - Q1 + v2 * cot * ir * ir, ap * irs - Q2};
            double hh[3] = {1.0, ir * ir, irs * irs};
#pragma unroll
            for (int a = 0; a < 3; a++) {
              m_[a] = (TC)mm[a];
              b2_[a] = (TC)(2.0 * beta[a]);
              h_[a] = (TC)(v2 * hh[a] - beta[a] * beta[a]);
            }
            bb_[0] = (TC)(2.0 * beta[0] * beta[1]);
            bb_[1] = (TC)(2.0 * beta[0] * beta[2]);
            bb_[2] = (TC)(2.0 * beta[1] * beta[2]);
          } else {
            // cylindrical x' = (r, phi, z): phi along the numerical y axis
            const double r = p.lo[0] + (i + 0.5) * p.dx[0];
            double sp, cp;
            trig_axis(p, 0, p.n[1] + 2 * PW_NG, j, sp, cp);
            double bv[3] = {ps.b[0], ps.b[1], ps.b[2]}, av[3] = {ps.a[0], ps.a[1], ps.a[2]};
            if (spin) {
              const double y[3] = {r * cp, r * sp, p.lo[2] + (k + 0.5) * p.dx[2]};
              frame_terms(ps, y, bv, av);
            }
            const double ir = 1.0 / r;
            const double br = cp * bv[0] + sp * bv[1], bp = cp * bv[1] - sp * bv[0];
            const double ar = cp * av[0] + sp * av[1], ap = cp * av[1] - sp * av[0];
            const double beta[3] = {br, bp * ir, bv[2]};
            const double Q0 = bp * bp * ir;
            const double Q1 = -2.0 * br * bp * ir * ir;
            const double mm[3] = {ar - Q0 + v2 * ir, ap * ir - Q1, av[2]};
            const double hh[3] = {1.0, ir * ir, 1.0};
#pragma unroll
            for (int a = 0; a < 3; a++) {
              m_[a] = (TC)mm[a];
              b2_[a] = (TC)(2.0 * beta[a]);
              h_[a] = (TC)(v2 * hh[a] - beta[a] * beta[a]);
            }
            bb_[0] = (TC)(2.0 * beta[0] * beta[1]);
            bb_[1] = (TC)(2.0 * beta[0] * beta[2]);
            bb_[2] = (TC)(2.0 * beta[1] * beta[2]);
          }
          const TC(*Bf)[ST_PW] = Bc[buf];
          // first derivatives of LDS plane F along x, y and of z-window row f along z
          auto ddx = [&](const TC *F) { return ((F[own - 2] - F[own + 2]) + (TC)8 * (F[own + 1] - F[own - 1])) * i12dx[0]; };
          auto ddy = [&](const TC *F) {
            return ((F[own - 2 * ST_PX] - F[own + 2 * ST_PX]) + (TC)8 * (F[own + ST_PX] - F[own - ST_PX])) * i12dx[1];
          };
          auto ddz = [&](int f) { return ((q[f][1] - q[f][5]) + (TC)8 * (q[f][4] - q[f][2])) * i12dx[2]; };
          TC dphi[3], d2phi[3], dpi[3], kof[5];
          if (FORM == 1) {
            // first-order form: Psi_a for D_a phi and D_a Psi_a for D_aa phi
#pragma unroll
            for (int a = 0; a < 3; a++) dphi[a] = q[2 + a][3];
            d2phi[0] = ddx(Bf[2]);
            d2phi[1] = ddy(Bf[3]);
            d2phi[2] = ddz(4);
          } else {
            const TC *F = Bf[0];
            TC u0 = F[own];
            TC xm1 = F[own - 1], xp1 = F[own + 1], xm2 = F[own - 2], xp2 = F[own + 2];
            TC ym1 = F[own - ST_PX], yp1 = F[own + ST_PX], ym2 = F[own - 2 * ST_PX], yp2 = F[own + 2 * ST_PX];
            TC zm1 = q[0][2], zp1 = q[0][4], zm2 = q[0][1], zp2 = q[0][5];
            dphi[0] = ((xm2 - xp2) + (TC)8 * (xp1 - xm1)) * i12dx[0];
            dphi[1] = ((ym2 - yp2) + (TC)8 * (yp1 - ym1)) * i12dx[1];
            dphi[2] = ((zm2 - zp2) + (TC)8 * (zp1 - zm1)) * i12dx[2];
            d2phi[0] = ((TC)16 * (xm1 + xp1) - (xm2 + xp2) - (TC)30 * u0) * i12dx2[0];
            d2phi[1] = ((TC)16 * (ym1 + yp1) - (ym2 + yp2) - (TC)30 * u0) * i12dx2[1];
            d2phi[2] = ((TC)16 * (zm1 + zp1) - (zm2 + zp2) - (TC)30 * u0) * i12dx2[2];
          }
          {
            const TC *F = Bf[1];
            dpi[0] = ((F[own - 2] - F[own + 2]) + (TC)8 * (F[own + 1] - F[own - 1])) * i12dx[0];
            dpi[1] = ((F[own - 2 * ST_PX] - F[own + 2 * ST_PX]) + (TC)8 * (F[own + ST_PX] - F[own - ST_PX])) * i12dx[1];
            dpi[2] = ((q[1][1] - q[1][5]) + (TC)8 * (q[1][4] - q[1][2])) * i12dx[2];
          }
#pragma unroll
          for (int f = 0; f < 5; f++) {
            const TC *F = Bf[f];
            const TC u0 = q[f][3];
            TC kx = (F[own - 3] + F[own + 3]) - (TC)6 * (F[own - 2] + F[own + 2]) + (TC)15 * (F[own - 1] + F[own + 1]) -
                    (TC)20 * u0;
            TC kyv = (F[own - 3 * ST_PX] + F[own + 3 * ST_PX]) - (TC)6 * (F[own - 2 * ST_PX] + F[own + 2 * ST_PX]) +
                     (TC)15 * (F[own - ST_PX] + F[own + ST_PX]) - (TC)20 * u0;
            TC kz = (q[f][0] + q[f][6]) - (TC)6 * (q[f][1] + q[f][5]) + (TC)15 * (q[f][2] + q[f][4]) - (TC)20 * u0;
            kof[f] = kx * ko[0] + kyv * ko[1] + kz * ko[2];
          }
          TC rhs_pi = (TC)0;
#pragma unroll
          for (int a = 0; a < 3; a++) rhs_pi += m_[a] * dphi[a] + b2_[a] * dpi[a] + h_[a] * d2phi[a];
          if (moving && FORM == 1) {
            // g^{ij} D_i Psi_j: the off-diagonal pairs enter as (D_i Psi_j + D_j Psi_i) / 2
            const TC sxy = ddx(Bf[3]) + ddy(Bf[2]);
            const TC sxz = ddx(Bf[4]) + ddz(2);
            const TC syz = ddy(Bf[4]) + ddz(3);
            rhs_pi -= (TC)0.5 * (bb_[0] * sxy + bb_[1] * sxz + bb_[2] * syz);
          } else if (moving) {
            const TC *F = Bf[0];
            TC sxy = (TC)0;
#pragma unroll
            for (int o2 = 0; o2 < 5; o2++) {
              if (o2 == 2) continue;
              TC inner = (TC)0;
#pragma unroll
              for (int o1 = 0; o1 < 5; o1++) {
                if (o1 == 2) continue;
                inner += w1[o1] * F[own + (o1 - 2) + (o2 - 2) * ST_PX];
              }
              sxy += w1[o2] * inner;
            }
            TC dxy = sxy * i12dx[0] * i12dx[1];
            TC sxz = (TC)0, syz = (TC)0;
#pragma unroll
            for (int o = 0; o < 5; o++) {
              sxz += w1[o] * dqx[o];
              syz += w1[o] * dqy[o];
            }
            TC dxz = sxz * i12dx[2], dyz = syz * i12dx[2];
            rhs_pi -= bb_[0] * dxy + bb_[1] * dxz + bb_[2] * dyz;
          }
          TC K[5];
          K[0] = q[1][3] + kof[0];
          K[1] = rhs_pi + kof[1];
#pragma unroll
          for (int a = 0; a < 3; a++) K[2 + a] = dpi[a] + kof[2 + a];
          const uint32_t x0 = col + (uint32_t)k * sz;
          // classic RK4 (Table rk4): v_{s+1} = u_n + a_s dt K_s; acc holds
          // u_n + dt sum_l b_l K_l in FP64, or (FP32 increments) dt sum_l b_l K_l in
          // FP32 with u_{n+1} = u_n + increment + b_4 dt K_4 formed in FP64.
#pragma unroll
          for (int f = 0; f < 5; f++) {
            const uint32_t x = f * fs + x0;
            if (INC) {
              const float kf = (float)K[f];
              if (STAGE == 0) {
                gst(AccF, x, bdtf * kf);
                gst(vout, x, (TOUT)((float)q[f][3] + adtf * kf));
              } else if (STAGE == 3) {
                const double un = cu[f] + ((double)cd[f] + bdt * (double)kf);
                gst(U, x, un);
                gst(Us, x, (float)un);
              } else {
                gst(AccF, x, cd[f] + bdtf * kf);
                gst(vout, x, (TOUT)(cus[f] + adtf * kf));
              }
            } else if (MIX) {
              const double kd = (double)K[f];
              if (STAGE == 0) {
                gst(Acc, x, cu[f] + bdt * kd);
                gst(vout, x, (TOUT)(cu[f] + adt * kd));
              } else if (STAGE == 3) {
                const double un = ca[f] + bdt * kd;
                gst(U, x, un);
                gst(Us, x, (float)un);
              } else {
                gst(Acc, x, ca[f] + bdt * kd);
                gst(vout, x, (TOUT)(cus[f] + adtf * (float)K[f]));
              }
            } else {
              const double kf = (double)K[f];
              if (STAGE == 0) {
                gst(Acc, x, cu[f] + bdt * kf);
                gst(vout, x, (TOUT)(cu[f] + adt * kf));
              } else if (STAGE == 3) {
                gst(U, x, ca[f] + bdt * kf);
              } else {
                gst(Acc, x, ca[f] + bdt * kf);
                gst(vout, x, (TOUT)(cu[f] + adt * kf));
              }
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Sommerfeld outer boundary (variant of the analytic outer boundary): every
// outer ghost cell of the global patch is evolved, with the same RK4 stage
// update as an interior cell, by the radiative condition for waves leaving the
// origin, d_t u = -v (X.grad u + u) / r on each field.  Derivatives: 4th-order
// centred along axes where the cell is interior, 2nd-order one-sided (inward)
// along axes where it is a ghost.  One thread per cell of the list.
// ---------------------------------------------------------------------------
template <typename TIN, typename TOUT, int STAGE, int AM>
__global__ void k_radiative(const PatchDev *__restrict__ P, const GhostRec *list, int count, int sv, double dt,
                            double v) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const PatchDev &p = P[0];
  if (!(p.sv_mask & (1u << sv))) return;
  int c[3];
  unpack_ijk(list[q].cell, c[0], c[1], c[2]);
  const TIN *in = (const TIN *)(STAGE == 0 ? (sizeof(TIN) == 8 ? (const void *)p.u[sv] : (const void *)p.us[sv])
                                           : (STAGE == 2 ? p.vb[sv] : p.va[sv]));
  TOUT *vout = (TOUT *)(STAGE == 1 ? p.vb[sv] : p.va[sv]);
  double *U = p.u[sv];
  double *Acc = p.acc[sv];
  float *AccF = (float *)p.acc[sv];
  float *Us = p.us[sv];
  constexpr bool MIX = sizeof(TOUT) == 4;
  constexpr bool INC = MIX && AM == 1;
  const double X[3] = {xnum(p, 0, c[0]), xnum(p, 1, c[1]), xnum(p, 2, c[2])};
  const double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  const long long x0 = cell_index(p, c[0], c[1], c[2]);
  const long long st[3] = {1, p.pitch, p.slab};
  double K[5], u0[5];
  for (int f = 0; f < 5; f++) {
    const TIN *F = in + f * p.fstride + x0;
    u0[f] = (double)F[0];
    double xgrad = 0.0;
    for (int a = 0; a < 3; a++) {
      const long long e = st[a];
      double d;
      if (c[a] < 0)
        d = (-3.0 * (double)F[0] + 4.0 * (double)F[e] - (double)F[2 * e]) / (2.0 * p.dx[a]);
      else if (c[a] >= p.n[a])
        d = (3.0 * (double)F[0] - 4.0 * (double)F[-e] + (double)F[-2 * e]) / (2.0 * p.dx[a]);
      else
        d = ((double)F[-2 * e] - 8.0 * (double)F[-e] + 8.0 * (double)F[e] - (double)F[2 * e]) / (12.0 * p.dx[a]);
      xgrad += X[a] * d;
    }
    K[f] = -v * (xgrad + u0[f]) / r;
  }
  // the stage update of k_stage (classic RK4, Table rk4) for this cell
  const double bdt = STAGE == 0 ? dt / 6.0 : (STAGE == 3 ? dt / 6.0 : dt / 3.0);
  const double adt = STAGE == 2 ? dt : dt / 2.0;
  const float bdtf = (float)bdt, adtf = (float)adt;
  for (int f = 0; f < 5; f++) {
    const long long x = f * p.fstride + x0;
    if (INC) {
      const float kf = (float)K[f];
      if (STAGE == 0) {
        AccF[x] = bdtf * kf;
        vout[x] = (TOUT)((float)u0[f] + adtf * kf);
      } else if (STAGE == 3) {
        const double un = U[x] + ((double)AccF[x] + bdt * (double)kf);
        U[x] = un;
        Us[x] = (float)un;
      } else {
        AccF[x] = AccF[x] + bdtf * kf;
        vout[x] = (TOUT)(Us[x] + adtf * kf);
      }
    } else if (MIX) {
      if (STAGE == 0) {
        Acc[x] = U[x] + bdt * K[f];
        vout[x] = (TOUT)(U[x] + adt * K[f]);
      } else if (STAGE == 3) {
        const double un = Acc[x] + bdt * K[f];
        U[x] = un;
        Us[x] = (float)un;
      } else {
        Acc[x] = Acc[x] + bdt * K[f];
        vout[x] = (TOUT)(Us[x] + adtf * (float)K[f]);
      }
    } else {
      if (STAGE == 0) {
        Acc[x] = U[x] + bdt * K[f];
        vout[x] = (TOUT)(U[x] + adt * K[f]);
      } else if (STAGE == 3) {
        U[x] = Acc[x] + bdt * K[f];
      } else {
        Acc[x] = Acc[x] + bdt * K[f];
        vout[x] = (TOUT)(U[x] + adt * K[f]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Utilities: fills, interior pack/unpack, exact initial data, diagnostics
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill_value(T *ptr, long long n, T val) {
  long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; q < n; q += (long long)gridDim.x * blockDim.x) ptr[q] = val;
}

// sin and cos of the grid angles of a curvilinear patch (see PatchDev::trig;
// a cylindrical patch uses the axis-1 entries only).
__global__ void k_trig_table(int n1, int n2, double lo1, double dx1, double lo2, double dx2, double *tab) {
  const int t1 = n1 + 2 * PW_NG, t2 = n2 + 2 * PW_NG;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < t1) {
    double sn, cs;
    sincos(lo1 + ((q - PW_NG) + 0.5) * dx1, &sn, &cs);
    tab[q] = sn;
    tab[t1 + q] = cs;
  } else if (q < t1 + t2) {
    double sn, cs;
    sincos(lo2 + ((q - t1 - PW_NG) + 0.5) * dx2, &sn, &cs);
    tab[2 * t1 + (q - t1)] = sn;
    tab[2 * t1 + t2 + (q - t1)] = cs;
  }
}

__global__ void k_unpack(const PatchDev *P, int pid, int sv, const double *src) {
  const PatchDev &p = P[pid];
  long long per = (long long)p.n[0] * p.n[1] * p.n[2];
  long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 5 * per) return;
  int f = (int)(q / per);
  long long c = q % per;
  int i = (int)(c % p.n[0]), j = (int)((c / p.n[0]) % p.n[1]), k = (int)(c / ((long long)p.n[0] * p.n[1]));
  const long long x = f * p.fstride + cell_index(p, i, j, k);
  p.u[sv][x] = src[q];
  if (p.us[sv]) p.us[sv][x] = (float)src[q];
}

__global__ void k_pack(const PatchDev *P, int pid, int sv, double *dst, int full) {
  const PatchDev &p = P[pid];
  int m0 = full ? p.n[0] + 2 * PW_NG : p.n[0], m1 = full ? p.n[1] + 2 * PW_NG : p.n[1],
      m2 = full ? p.n[2] + 2 * PW_NG : p.n[2];
  int off = full ? -PW_NG : 0;
  long long per = (long long)m0 * m1 * m2;
  long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 5 * per) return;
  int f = (int)(q / per);
  long long c = q % per;
  int i = (int)(c % m0) + off, j = (int)((c / m0) % m1) + off, k = (int)(c / ((long long)m0 * m1)) + off;
  dst[q] = p.u[sv][f * p.fstride + cell_index(p, i, j, k)];
}

__global__ void k_init_exact(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, int pid, int sv, const ExactDev *ex, double v,
                             double t) {
  const PatchDev &p = P[pid];
  long long per = (long long)p.n[0] * p.n[1] * p.n[2];
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= per) return;
  int i = (int)(c % p.n[0]), j = (int)((c / p.n[0]) % p.n[1]), k = (int)(c / ((long long)p.n[0] * p.n[1]));
  double xp[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)}, e[5];
  exact_patch(ex[sv], v, p, pose[pid], t, xp, e);
  long long x = cell_index(p, i, j, k);
  for (int f = 0; f < 5; f++) p.u[sv][f * p.fstride + x] = e[f];
  if (p.us[sv])
    for (int f = 0; f < 5; f++) p.us[sv][f * p.fstride + x] = (float)e[f];
}

// Per-block partial diagnostics: 23 doubles per block (see pw_diag).
__global__ void k_diag(const PatchDev *__restrict__ P, const PoseDev *__restrict__ pose, int pid, int sv, const uint8_t *gflag,
                       const ExactDev *ex, double v, double t, double *partial) {
  const PatchDev &p = P[pid];
  long long per = (long long)p.n[0] * p.n[1] * p.n[2];
  __shared__ double red[256][DIAG_N];
  double acc[DIAG_N];
  for (int x = 0; x < DIAG_N; x++) acc[x] = 0.0;
  const bool has = ex[sv].kind != EX_NONE;
  const double cellvol = p.dx[0] * p.dx[1] * p.dx[2];
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < per; c += (long long)gridDim.x * blockDim.x) {
    if (p.is_global && gflag && gflag[c] != LIVE) continue;
    int i = (int)(c % p.n[0]), j = (int)((c / p.n[0]) % p.n[1]), k = (int)(c / ((long long)p.n[0] * p.n[1]));
    double xp[3] = {xnum(p, 0, i), xnum(p, 1, j), xnum(p, 2, k)}, e[5] = {0, 0, 0, 0, 0};
    if (has) exact_patch(ex[sv], v, p, pose[pid], t, xp, e);
    long long x = cell_index(p, i, j, k);
    double phi = 0;
    for (int f = 0; f < 5; f++) {
      double val = p.u[sv][f * p.fstride + x];
      if (f == 0) phi = val;
      acc[f] = fmax(acc[f], fabs(val));
      acc[5 + f] += val * val;
      if (has) {
        double d = val - e[f];
        acc[10 + f] = fmax(acc[10 + f], fabs(d));
        acc[15 + f] += d * d;
      }
    }
    double sg = p.coord == CART ? 1.0 : p.coord == SPH ? xp[0] * xp[0] * fabs(sin(xp[1])) : xp[0];
    if (has) acc[20] += fabs(phi - e[0]) / fabs(e[0]) * sg * cellvol;
    acc[21] += 1.0;
    acc[22] += sg * cellvol;
    // energy density 1/2 (Pi_t^2 - v^2 phi L phi) and the constraint Psi_a - D_a phi,
    // where the +-2 axis stencils reach live interior cells only (periodic axes wrap)
    double ph[3][5];
    bool ok = true;
    const int ci[3] = {i, j, k};
    for (int a = 0; a < 3 && ok; a++)
      for (int o = -2; o <= 2 && ok; o++) {
        int cc[3] = {ci[0], ci[1], ci[2]};
        cc[a] += o;
        if (p.periodic[a]) cc[a] = ((cc[a] % p.n[a]) + p.n[a]) % p.n[a];
        if (cc[a] < 0 || cc[a] >= p.n[a]) {
          ok = false;
          break;
        }
        if (p.is_global && gflag && gflag[((long long)cc[2] * p.n[1] + cc[1]) * p.n[0] + cc[0]] != LIVE) {
          ok = false;
          break;
        }
        ph[a][o + 2] = p.u[sv][cell_index(p, cc[0], cc[1], cc[2])];
      }
    if (ok) {
      double lap = 0.0;
      for (int a = 0; a < 3; a++) {
        lap += (-ph[a][0] + 16.0 * ph[a][1] - 30.0 * ph[a][2] + 16.0 * ph[a][3] - ph[a][4]) /
               (12.0 * p.dx[a] * p.dx[a]);
        const double d1 = (ph[a][0] - 8.0 * ph[a][1] + 8.0 * ph[a][3] - ph[a][4]) / (12.0 * p.dx[a]);
        acc[24 + a] = fmax(acc[24 + a], fabs(p.u[sv][(2 + a) * p.fstride + x] - d1));
      }
      const double pit = p.u[sv][p.fstride + x];
      acc[23] += 0.5 * cellvol * (pit * pit - v * v * ph[0][2] * lap);
    }
  }
  for (int x = 0; x < DIAG_N; x++) red[threadIdx.x][x] = acc[x];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int x = 0; x < DIAG_N; x++) {
        bool mx = (x < 5) || (x >= 10 && x < 15) || x >= 24;
        double o = red[threadIdx.x + s][x];
        red[threadIdx.x][x] = mx ? fmax(red[threadIdx.x][x], o) : red[threadIdx.x][x] + o;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int x = 0; x < DIAG_N; x++) partial[(long long)blockIdx.x * DIAG_N + x] = red[0][x];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_pose(hipStream_t s, const PatchDev *P, int np, const double *tdev, double dt, PoseDev *poses) {
  hipLaunchKernelGGL(k_pose, dim3(nblk(np, 64)), dim3(64), 0, s, P, np, tdev, dt, poses);
}
void launch_pose_at(hipStream_t s, const PatchDev *P, int np, double t, PoseDev *out) {
  hipLaunchKernelGGL(k_pose_at, dim3(nblk(np, 64)), dim3(64), 0, s, P, np, t, out);
}
void launch_advance_time(hipStream_t s, double *tdev, double dt, long long *counters) {
  hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, s, tdev, dt, counters);
}

// The chunked filters apply: rows of a multiple of 16 cells, arrays 16-byte aligned.
static bool chunked(int n0, std::initializer_list<const void *> ptrs) {
  if (n0 % 16 != 0) return false;
  for (const void *p : ptrs)
    if ((uintptr_t)p % 16 != 0) return false;
  return true;
}

void launch_flags(hipStream_t s, const FlagsArgs &a) {
  const int bs = 256;
  long long tot = (long long)a.n[0] * a.n[1] * a.n[2];
  unsigned nb = nblk(tot, bs);
  const dim3 g3(nblk(a.n[0], bs), a.n[1], a.n[2]);
  hipLaunchKernelGGL(k_fill_value<uint8_t>, dim3(nb < 4096 ? nb : 4096), dim3(bs), 0, s, a.dbl, tot, (uint8_t)0);
  if (a.nblks > 0)
    hipLaunchKernelGGL(k_cover, dim3(a.nblks), dim3(256), 0, s, a.P, a.pose, a.jobs, a.blks, a.cover_new,
                       a.dbl);
  if (a.nphys > 0) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, a.ocount, 0);
    hipLaunchKernelGGL(k_cover_outer, dim3(nblk(a.nphys, 256)), dim3(256), 0, s, a.P, a.pose, a.jobs, a.njobs,
                       a.phys, a.nphys, a.olist, a.ocount);
  }
  if (chunked(a.n[0], {a.cover_new, a.t1, a.t2, a.live, a.flag_new, a.dbl}) && a.buffer <= 4 && PW_NG <= 4) {
    // live = buffer-dilation of the uncovered cells, near = NG-dilation of live
    const dim3 gc(nblk((long long)(a.n[0] / 16) * a.n[1], bs), a.n[2]);
    hipLaunchKernelGGL(k_dilate_x16<true>, gc, dim3(bs), 0, s, (const void *)a.cover_new, a.t1, a.n[0], a.n[1],
                       a.buffer, 1, a.wrap[0]);
    hipLaunchKernelGGL((k_dilate_yz16<1, false>), gc, dim3(bs), 0, s, (const uint8_t *)a.t1, a.t2, a.n[0], a.n[1],
                       a.n[2], a.buffer, 1, a.wrap[1], nullptr, nullptr, nullptr);
    hipLaunchKernelGGL((k_dilate_yz16<2, false>), gc, dim3(bs), 0, s, (const uint8_t *)a.t2, a.live, a.n[0], a.n[1],
                       a.n[2], a.buffer, 1, a.wrap[2], nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_dilate_x16<false>, gc, dim3(bs), 0, s, (const void *)a.live, a.t1, a.n[0], a.n[1], PW_NG,
                       0, a.wrap[0]);
    hipLaunchKernelGGL((k_dilate_yz16<1, false>), gc, dim3(bs), 0, s, (const uint8_t *)a.t1, a.t2, a.n[0], a.n[1],
                       a.n[2], PW_NG, 0, a.wrap[1], nullptr, nullptr, nullptr);
    hipLaunchKernelGGL((k_dilate_yz16<2, true>), gc, dim3(bs), 0, s, (const uint8_t *)a.t2, a.flag_new, a.n[0],
                       a.n[1], a.n[2], PW_NG, 0, a.wrap[2], (const uint8_t *)a.live, (const uint8_t *)a.dbl, a.err);
    return;
  }
  hipLaunchKernelGGL((k_dilate<0, true>), g3, dim3(bs), 0, s, (const void *)a.cover_new, a.t1, a.n[0], a.n[1],
                     a.n[2], a.buffer, 1, a.wrap[0]);
  hipLaunchKernelGGL((k_dilate<1, false>), g3, dim3(bs), 0, s, (const void *)a.t1, a.t2, a.n[0], a.n[1], a.n[2],
                     a.buffer, 1, a.wrap[1]);
  hipLaunchKernelGGL((k_dilate<2, false>), g3, dim3(bs), 0, s, (const void *)a.t2, a.live, a.n[0], a.n[1],
                     a.n[2], a.buffer, 1, a.wrap[2]);
  hipLaunchKernelGGL((k_dilate<0, false>), g3, dim3(bs), 0, s, (const void *)a.live, a.t1, a.n[0], a.n[1],
                     a.n[2], PW_NG, 0, a.wrap[0]);
  hipLaunchKernelGGL((k_dilate<1, false>), g3, dim3(bs), 0, s, (const void *)a.t1, a.t2, a.n[0], a.n[1], a.n[2],
                     PW_NG, 0, a.wrap[1]);
  hipLaunchKernelGGL((k_dilate<2, false>), g3, dim3(bs), 0, s, (const void *)a.t2, a.t1, a.n[0], a.n[1], a.n[2],
                     PW_NG, 0, a.wrap[2]);
  hipLaunchKernelGGL(k_combine_flags, dim3(nb), dim3(bs), 0, s, (const uint8_t *)a.live, (const uint8_t *)a.t1,
                     (const uint8_t *)a.dbl, a.flag_new, tot, a.err);
}

void launch_l2g_order(hipStream_t s, const L2GOrderArgs &a) {
  if (a.nbuckets <= 0) return;
  hipLaunchKernelGGL(k_fill_value<int>, dim3(nblk(a.nbuckets, 256) < 4096 ? nblk(a.nbuckets, 256) : 4096), dim3(256), 0,
                     s, a.cnt, (long long)a.nbuckets, 0);
  hipLaunchKernelGGL(k_bucket_count, dim3(1024), dim3(256), 0, s, a.P, a.pose, (const int32_t *)a.list, a.count,
                     a.cover, a.rank, a.cnt, a.ebkt, a.erank);
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, (const int *)a.cnt, a.off, a.nbuckets);
  hipLaunchKernelGGL(k_bucket_scatter, dim3(1024), dim3(256), 0, s, (const int32_t *)a.list, a.count,
                     (const int *)a.ebkt, (const int *)a.erank, (const int *)a.off, a.sorted);
  hipLaunchKernelGGL(k_bucket_sort, dim3(a.nbuckets), dim3(256), 0, s, (const int32_t *)a.sorted, (const int *)a.cnt,
                     (const int *)a.off, a.nbuckets, a.out);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, a.nitems, 0);
  hipLaunchKernelGGL(k_l2g_items, dim3(nblk(a.nbuckets, 256)), dim3(256), 0, s, (const int *)a.cnt,
                     (const int *)a.off, a.nbuckets, a.items, a.nitems);
}

void launch_finalize(hipStream_t s, const FinalizeArgs &a) {
  long long tot = (long long)a.n[0] * a.n[1] * a.n[2];
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, a.ucount, 0);
  hipLaunchKernelGGL(k_finalize, dim3(nblk((tot + FIN_CELLS - 1) / FIN_CELLS, 256)), dim3(256), 0, s, a.P, a.flag_cur,
                     a.flag_new, a.cover_cur, a.cover_new, a.nsv, a.mode, a.ulist, a.ucount);
  if (a.mode == 1)
    hipLaunchKernelGGL(k_uncover, dim3(64), dim3(256), 0, s, a.P, a.pose, (const int2 *)a.ulist,
                       (const int *)a.ucount, (const int32_t *)a.cover_cur, a.nsv, a.Pts, a.ex, a.vs, a.tdev,
                       a.counters);
  if (a.nphys > 0)
    hipLaunchKernelGGL(k_copy_olist, dim3(64), dim3(256), 0, s, a.olist_new, a.ocount_new, a.olist_cur,
                       a.ocount_cur);
}

template <typename TB, typename TC>
static void ghosts_typed(hipStream_t s, const GhostArgs &a) {
  const int bs = 256;
  const int l0 = (a.parts & GH_GLOBAL) ? 0 : a.n_lower_global;
  const int l1 = (a.parts & GH_LOCAL) ? a.n_lower : a.n_lower_global;
  const bool g2l = a.n_bricks > 0 && (a.parts & GH_LOCAL);
  const bool l2g = a.has_locals && (a.parts & GH_GLOBAL);
  // the lower-priority fill (outer ghosts, periodic copies) comes last: the
  // periodic copies of a spherical global then carry the effective ghosts'
  // interpolated values; nothing in the interpatch fills reads these cells
  auto lower = [&]() {
    // the global entries are skipped when an earlier stage at the same time wrote them already
    const int lb = a.lower_skip_global && l0 < a.n_lower_global ? a.n_lower_global : l0;
    if (l1 > lb)
      hipLaunchKernelGGL(k_fill_lower<TB>, dim3(nblk(l1 - lb, bs)), dim3(bs), 0, s, a.P, a.pose, a.lower + lb,
                         l1 - lb, a.sv, a.stage, a.ex, a.v, a.tdev, a.tmul, a.dt, a.lower_dup);
    // covered physical ghosts of the global patch: interpatch over the boundary value
    if ((a.parts & GH_GLOBAL) && a.olist)
      hipLaunchKernelGGL((k_l2g_outer<TB, TC>), dim3(std::min(1024u, nblk(a.nphys, 256))), dim3(256), 0, s, a.P,
                         a.pose, a.phys, a.olist, a.ocount,
                         a.sv, a.stage, a.Pts, a.skips);
  };
  if (!g2l && !l2g) {
    if (a.phases & PH_LOWER) lower();
    return;
  }
  auto run_g2l = [&]() {
    if (a.g2l_exact_only) {
      hipLaunchKernelGGL(k_g2l_exact<TB>, dim3(a.n_bricks), dim3(BRICK_THREADS), 0, s, a.P, a.pose, a.bricks,
                         a.n_bricks, a.sv, a.stage, a.ex, a.v, a.tdev, a.tmul, a.dt);
      return;
    }
    if (a.global_curv) {
      hipLaunchKernelGGL((k_g2l_point<TB, TC>), dim3(a.n_bricks), dim3(BRICK_THREADS), 0, s, a.P, a.pose, a.bricks,
                         a.n_bricks, a.sv, a.stage, a.gflag, a.l2g_first, a.Pts, a.skips, a.fb, a.fb_count);
      return;
    }
    const int run = a.g2l_run;
    const int bchunk = (a.n_bricks + 8 * run - 1) / (8 * run);
    const dim3 g(8 * run * bchunk), b(BRICK_THREADS);
#define PW_G2L(PP)                                                                                           \
  hipLaunchKernelGGL((k_g2l_brick<TB, TC, PP>), g, b, 0, s, a.P, a.pose, a.bricks, a.n_bricks, run, a.sv, a.stage, \
                     a.dvalid, a.skips, a.fb, a.fb_count)
    switch (a.Pts) {
      case 2: PW_G2L(2); break;
      case 3: PW_G2L(3); break;
      case 4: PW_G2L(4); break;
      case 5: PW_G2L(5); break;
      default: PW_G2L(6); break;
    }
#undef PW_G2L
  };
  auto run_l2g = [&]() {
    if (a.global_curv) {
      hipLaunchKernelGGL((k_l2g_point<TB, TC>), dim3(1024), dim3(256), 0, s, a.P, a.pose, a.efflist, a.effcount,
                         a.cover, a.sv, a.stage, a.Pts, a.skips + 1, a.fb, a.fb_count);
      return;
    }
    const dim3 g(L2G_BLOCKS), b(L2G_THREADS);
#define PW_L2G(PP)                                                                                                \
  hipLaunchKernelGGL((k_l2g_bucket<TB, TC, PP>), g, b, 0, s, a.P, a.pose, a.efflist, a.l2g_items, a.l2g_nitems,   \
                     a.l2g_run, a.cover, a.sv, a.stage, a.skips + 1, a.fb, a.fb_count, a.l2g_direct)
    switch (a.Pts) {
      case 2: PW_L2G(2); break;
      case 3: PW_L2G(3); break;
      case 4: PW_L2G(4); break;
      case 5: PW_L2G(5); break;
      default: PW_L2G(6); break;
    }
#undef PW_L2G
  };
  auto fallback = [&]() {
    hipLaunchKernelGGL(k_fallback<TB>, dim3(64), dim3(256), 0, s, a.P, a.pose, a.fb, a.fb_count, a.sv, a.stage, a.ex,
                       a.v, a.tdev, a.tmul, a.dt);
  };
  if (a.l2g_first && g2l && l2g) {
    // narrow buffer: the effective ghosts (with their fallbacks) are complete
    // before the global -> local stencils read them
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, a.fb_count, 0);
    run_l2g();
    fallback();
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, a.fb_count, 0);
    run_g2l();
    fallback();
    lower();
    return;
  }
  if (a.phases & PH_INTERP) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, a.fb_count, 0);
    if (g2l) run_g2l();
    if (l2g) run_l2g();
  }
  if (a.phases & PH_FALLBACK) fallback();
  if (a.phases & PH_LOWER) lower();
}

void launch_ghosts(hipStream_t s, const GhostArgs &a) {
  if (a.stage_fp64) {
    if (a.mixed) ghosts_typed<double, float>(s, a);
    else ghosts_typed<double, double>(s, a);
  } else {
    ghosts_typed<float, float>(s, a);
  }
}

void launch_post_flags(hipStream_t s, const PostFlagsArgs &a) {
  // (the donor ordering of the list is done by launch_l2g_order after this)
  const dim3 g3(nblk(a.n[0], 256), a.n[1], a.n[2]);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, a.effcount, 0);
  const long long tot_bricks = (long long)((a.n[0] + 3) / 4) * ((a.n[1] + 3) / 4) * ((a.n[2] + 3) / 4) * 64;
  hipLaunchKernelGGL(k_efflist, dim3(nblk(tot_bricks, 256 * EFF_PER_THREAD)), dim3(256), 0, s,
                     (const uint8_t *)a.flag, a.n[0], a.n[1], a.n[2], a.efflist, a.effcount);
  const bool ck = chunked(a.n[0], {a.flag, a.t1, a.t2});
  const dim3 gc(nblk((long long)(a.n[0] / 16) * a.n[1], 256), a.n[2]);
  for (int m = 0; m < PW_NPTS; m++) {
    if (!a.dvalid[m]) continue;
    int P = a.Pvals[m];
    if (ck && P <= 8 && chunked(a.n[0], {a.dvalid[m]})) {
      hipLaunchKernelGGL(k_window_x16, gc, dim3(256), 0, s, (const uint8_t *)a.flag, a.t1, a.n[0], a.n[1], P,
                         a.donor_effghost ? 2 : 1, a.wrap[0]);
      hipLaunchKernelGGL(k_window_yz16<1>, gc, dim3(256), 0, s, (const uint8_t *)a.t1, a.t2, a.n[0], a.n[1], a.n[2],
                         P, a.wrap[1]);
      hipLaunchKernelGGL(k_window_yz16<2>, gc, dim3(256), 0, s, (const uint8_t *)a.t2, a.dvalid[m], a.n[0], a.n[1],
                         a.n[2], P, a.wrap[2]);
      continue;
    }
    hipLaunchKernelGGL(k_window_min<0>, g3, dim3(256), 0, s, (const uint8_t *)a.flag, a.t1, a.n[0], a.n[1],
                       a.n[2], P, a.donor_effghost ? 2 : 1, a.wrap[0]);
    hipLaunchKernelGGL(k_window_min<1>, g3, dim3(256), 0, s, (const uint8_t *)a.t1, a.t2, a.n[0], a.n[1],
                       a.n[2], P, 0, a.wrap[1]);
    hipLaunchKernelGGL(k_window_min<2>, g3, dim3(256), 0, s, (const uint8_t *)a.t2, a.dvalid[m], a.n[0],
                       a.n[1], a.n[2], P, 0, a.wrap[2]);
  }
}

// One stage launch over tiles of one topology (global patch or local patches).
template <typename TIN, typename TOUT, typename TC, int ST, int AM, int FORM, int SH>
static void launch_stage_local(hipStream_t s, const StageArgs &a, dim3 g, int chunk) {
  const dim3 bs(StageTile<false, SH>::THREADS);
  if (a.coord == CART)
    hipLaunchKernelGGL((k_stage<TIN, TOUT, TC, ST, CART, false, AM, FORM, SH>), g, bs, 0, s, a.P, a.pose, a.tiles,
                       a.ntiles, chunk, a.gflag, a.sv, a.dt, a.v2, a.eps);
  else if (a.coord == SPH)
    hipLaunchKernelGGL((k_stage<TIN, TOUT, TC, ST, SPH, false, AM, FORM, SH>), g, bs, 0, s, a.P, a.pose, a.tiles,
                       a.ntiles, chunk, a.gflag, a.sv, a.dt, a.v2, a.eps);
  else
    hipLaunchKernelGGL((k_stage<TIN, TOUT, TC, ST, CYL, false, AM, FORM, SH>), g, bs, 0, s, a.P, a.pose, a.tiles,
                       a.ntiles, chunk, a.gflag, a.sv, a.dt, a.v2, a.eps);
}

template <typename TIN, typename TOUT, typename TC, int ST, int AM, int FORM, int SH>
static void launch_stage_global(hipStream_t s, const StageArgs &a, dim3 g, int chunk) {
  const dim3 bs(StageTile<true, SH>::THREADS);
  if (a.coord == CART)
    hipLaunchKernelGGL((k_stage<TIN, TOUT, TC, ST, CART, true, AM, FORM, SH>), g, bs, 0, s, a.P, a.pose, a.tiles,
                       a.ntiles, chunk, a.gflag, a.sv, a.dt, a.v2, a.eps);
  else  // a spherical global patch
    hipLaunchKernelGGL((k_stage<TIN, TOUT, TC, ST, SPH, true, AM, FORM, SH>), g, bs, 0, s, a.P, a.pose, a.tiles,
                       a.ntiles, chunk, a.gflag, a.sv, a.dt, a.v2, a.eps);
}

template <typename TIN, typename TOUT, typename TC, int ST, int AM, int FORM>
static void launch_stage_t(hipStream_t s, const StageArgs &a) {
  const int chunk = (a.ntiles + 7) / 8;
  const dim3 g(8 * chunk);
  if (a.global) {
    if (a.global_tile == 1) launch_stage_global<TIN, TOUT, TC, ST, AM, FORM, 1>(s, a, g, chunk);
    else if (sizeof(TC) == 4 && a.global_tile == 2)  // mixed modes only (FP64 would spill registers)
      launch_stage_global<TIN, TOUT, TC, ST, AM, FORM, (sizeof(TC) == 4 ? 2 : 1)>(s, a, g, chunk);
    else launch_stage_global<TIN, TOUT, TC, ST, AM, FORM, 0>(s, a, g, chunk);
  } else if (a.local_tile == 1) {
    launch_stage_local<TIN, TOUT, TC, ST, AM, FORM, 1>(s, a, g, chunk);
  } else {
    launch_stage_local<TIN, TOUT, TC, ST, AM, FORM, 0>(s, a, g, chunk);
  }
}

template <int FORM>
static void launch_stage_f(hipStream_t s, const StageArgs &a) {
  if (!a.mixed) {
    switch (a.stage) {
      case 0: launch_stage_t<double, double, double, 0, 0, FORM>(s, a); break;
      case 1: launch_stage_t<double, double, double, 1, 0, FORM>(s, a); break;
      case 2: launch_stage_t<double, double, double, 2, 0, FORM>(s, a); break;
      default: launch_stage_t<double, double, double, 3, 0, FORM>(s, a); break;
    }
  } else if (!a.inc) {
    switch (a.stage) {
      case 0: launch_stage_t<float, float, float, 0, 0, FORM>(s, a); break;
      case 1: launch_stage_t<float, float, float, 1, 0, FORM>(s, a); break;
      case 2: launch_stage_t<float, float, float, 2, 0, FORM>(s, a); break;
      default: launch_stage_t<float, float, float, 3, 0, FORM>(s, a); break;
    }
  } else {
    switch (a.stage) {
      case 0: launch_stage_t<float, float, float, 0, 1, FORM>(s, a); break;
      case 1: launch_stage_t<float, float, float, 1, 1, FORM>(s, a); break;
      case 2: launch_stage_t<float, float, float, 2, 1, FORM>(s, a); break;
      default: launch_stage_t<float, float, float, 3, 1, FORM>(s, a); break;
    }
  }
}

void launch_stage(hipStream_t s, const StageArgs &a) {
  if (a.ntiles <= 0) return;
  if (a.form == 1)
    launch_stage_f<1>(s, a);
  else
    launch_stage_f<0>(s, a);
}

template <typename TIN, typename TOUT, int AM>
static void launch_radiative_t(hipStream_t s, const PatchDev *P, const GhostRec *list, int count, int sv, int stage,
                               double dt, double v) {
  const dim3 g(nblk(count, 256)), b(256);
  switch (stage) {
    case 0: hipLaunchKernelGGL((k_radiative<TIN, TOUT, 0, AM>), g, b, 0, s, P, list, count, sv, dt, v); break;
    case 1: hipLaunchKernelGGL((k_radiative<TIN, TOUT, 1, AM>), g, b, 0, s, P, list, count, sv, dt, v); break;
    case 2: hipLaunchKernelGGL((k_radiative<TIN, TOUT, 2, AM>), g, b, 0, s, P, list, count, sv, dt, v); break;
    default: hipLaunchKernelGGL((k_radiative<TIN, TOUT, 3, AM>), g, b, 0, s, P, list, count, sv, dt, v); break;
  }
}

void launch_radiative(hipStream_t s, const PatchDev *P, const GhostRec *list, int count, int sv, int stage,
                      int mixed, int inc, double dt, double v) {
  if (count <= 0) return;
  if (!mixed)
    launch_radiative_t<double, double, 0>(s, P, list, count, sv, stage, dt, v);
  else if (!inc)
    launch_radiative_t<float, float, 0>(s, P, list, count, sv, stage, dt, v);
  else
    launch_radiative_t<float, float, 1>(s, P, list, count, sv, stage, dt, v);
}

void launch_fill_list(hipStream_t s, const PatchDev *P, const PoseDev *pose, const GhostRec *list, int count, int sv,
                      int fp64, const ExactDev *ex, double v, const double *tdev) {
  if (count <= 0) return;
  if (fp64)
    hipLaunchKernelGGL(k_fill_lower<double>, dim3(nblk(count, 256)), dim3(256), 0, s, P, pose, list, count, sv, 0, ex,
                       v, tdev, 0.0, 0.0, -1);
  else
    hipLaunchKernelGGL(k_fill_lower<float>, dim3(nblk(count, 256)), dim3(256), 0, s, P, pose, list, count, sv, 0, ex,
                       v, tdev, 0.0, 0.0, -1);
}

void launch_trig_table(hipStream_t s, int n1, int n2, double lo1, double dx1, double lo2, double dx2, double *tab) {
  const int n = n1 + n2 + 4 * PW_NG;
  hipLaunchKernelGGL(k_trig_table, dim3(nblk(n, 256)), dim3(256), 0, s, n1, n2, lo1, dx1, lo2, dx2, tab);
}
void launch_fill_f64(hipStream_t s, double *p, long long n, double v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_value<double>, dim3(nblk(n, 256) < 4096 ? nblk(n, 256) : 4096), dim3(256), 0, s, p, n, v);
}
void launch_fill_f32(hipStream_t s, float *p, long long n, float v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_value<float>, dim3(nblk(n, 256) < 4096 ? nblk(n, 256) : 4096), dim3(256), 0, s, p, n, v);
}
void launch_fill_i32(hipStream_t s, int32_t *p, long long n, int32_t v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_value<int32_t>, dim3(nblk(n, 256) < 4096 ? nblk(n, 256) : 4096), dim3(256), 0, s, p, n, v);
}
void launch_fill_u8(hipStream_t s, uint8_t *p, long long n, uint8_t v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_value<uint8_t>, dim3(nblk(n, 256) < 4096 ? nblk(n, 256) : 4096), dim3(256), 0, s, p, n, v);
}
void launch_unpack(hipStream_t s, const PatchDev *P, int pid, int sv, const double *src, long long n) {
  hipLaunchKernelGGL(k_unpack, dim3(nblk(n, 256)), dim3(256), 0, s, P, pid, sv, src);
}
void launch_pack(hipStream_t s, const PatchDev *P, int pid, int sv, double *dst, long long n, int full) {
  hipLaunchKernelGGL(k_pack, dim3(nblk(n, 256)), dim3(256), 0, s, P, pid, sv, dst, full);
}
void launch_init_exact(hipStream_t s, const PatchDev *P, const PoseDev *pose, int pid, int sv, const ExactDev *ex,
                       double v, double t, long long ncell) {
  hipLaunchKernelGGL(k_init_exact, dim3(nblk(ncell, 256)), dim3(256), 0, s, P, pose, pid, sv, ex, v, t);
}
void launch_diag(hipStream_t s, const PatchDev *P, const PoseDev *pose, int pid, int sv, const uint8_t *gflag,
                 const ExactDev *ex, double v, double t, double *partial, int nblocks) {
  hipLaunchKernelGGL(k_diag, dim3(nblocks), dim3(256), 0, s, P, pose, pid, sv, gflag, ex, v, t, partial);
}

}  // namespace pw
