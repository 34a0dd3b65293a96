// Level-0 pre-smoothing sweep fused with the restriction of the smoothed
// iterate's residual (Sec. 4.2: one block-Jacobi sweep, then R (f - A U')),
// for 2D periodic levels with a constant reaction or (FP32) a per-point
// reaction coefficient (the Newton linearization), space coarsening, and tiles of
// 32 x 8 coarse points that cover the coarse grid exactly.
//
// With the sweep U' = U + omega d, d = C^{-1} r, r = f - A U (C: the slab
// blocks B on the diagonal and -cin cout^T below it inside a chunk), the
// residual of U' needs no second stencil pass over U' (the reaction is
// pointwise, so a reaction coefficient sits in C's point blocks):
//   f - A U' = (1 - omega) r - omega (A - C) d,
//   (A - C) d = -db (cx (d_W + d_E) + cy (d_S + d_N)) - [chunk start] cin (cout . d_{n-1}),
// so a tile needs r on its points and d on their spatial neighbours.  One
// workgroup takes one tile and a run of whole smoother chunks; every
// thread smooths its 2 x 2 fine block and one point of the ring of 245
// fine points around the tile whose corrections the tile's residuals need
// (81 of them are also residual points of the restriction: the tile's left
// fine column and top fine row).  Per slab the corrections go to an LDS tile,
// the residuals of U' to a second one, and each thread restricts its coarse
// point (full weighting) and, with ZS, does the coarse level's first sweep
// from zero along its coarse chunks, as k_restrict_blk.
//
// Inside a run the chunk-start term takes cout . d of the previous slab from
// registers.  At the first slab of a run it needs cout . d of the previous
// run's last slab, which another workgroup computes: each run
// leaves cout . d of its last slab in zbuf, and k_sr_fixup adds
// omega cin R(cout . d) to the coarse right-hand side of that slab and the
// response of the coarse zero-guess sweep to it along the coarse chunk it
// starts (the sweep is linear in its right-hand side).
#include "kernels_impl.hpp"

namespace stmg {
namespace {

constexpr int kSrTCX = 32, kSrTCY = 8;                 // coarse points per tile
constexpr int kSrFX = 2 * kSrTCX, kSrFY = 2 * kSrTCY;  // fine points per tile
constexpr int kSrDW = kSrFX + 3, kSrDH = kSrFY + 3;    // correction tile, fine x, y in [-2, 64] x [-2, 16]
constexpr int kSrRW = 2 * (kSrTCX + 1);                // residual tile row: even then odd columns
constexpr int kSrRH = kSrFY + 1;                       // residual tile rows, fine y in [-1, 15]
constexpr int kSrRing = 245;
constexpr int kSrMaxCs = 8;  // coarse chunk lengths the fix-up takes
constexpr int kSrRHalo = 81;
static_assert(kSrTCX * kSrTCY == kBlock, "one coarse point per thread");
static_assert(kSrRing <= kBlock, "one ring point per thread");

// Ring point t (tile-local fine coordinates, the tile's own points are
// [0, 64) x [0, 16)): 0..16 column -1 (rows -1..15), 17..80 row -1 (columns
// 0..63), 81..82 column -1 rows -2 and 16, 83..99 column -2, 100..116 column
// 64 (rows -1..15), 117..180 row -2, 181..244 row 16 (columns 0..63).
__device__ __forceinline__ void sr_ring_point(int t, int& lx, int& ly) {
  if (t < 17) { lx = -1; ly = t - 1; }
  else if (t < 81) { lx = t - 17; ly = -1; }
  else if (t < 83) { lx = -1; ly = t == 81 ? -2 : kSrFY; }
  else if (t < 100) { lx = -2; ly = t - 84; }
  else if (t < 117) { lx = kSrFX; ly = t - 101; }
  else if (t < 181) { lx = t - 117; ly = -2; }
  else { lx = t - 181; ly = kSrFY; }
}

template <int M, typename T, int REACT, bool ZS, bool HASF>
__global__ __launch_bounds__(kBlock) void k_smooth_restrict(const OpParams p, const SweepPtrs<T> a, int ncx,
                                                            int ncy, T* __restrict__ fc, int RL, int chunk, int tiles_x,
                                                            int tiles, int nblocks, const OpParams pc,
                                                            T* __restrict__ uc, const T* __restrict__ coefc, int cs,
                                                            T* __restrict__ zbuf) {
  __shared__ T Dt[M * kSrDH * kSrDW];
  __shared__ T Rt[M * kSrRH * kSrRW];
  auto dt = [&](int i, int ly, int lx) -> T& { return Dt[(i * kSrDH + ly + 2) * kSrDW + lx + 2]; };
  auto rt = [&](int i, int y, int x) -> T& { return Rt[(i * kSrRH + y) * kSrRW + (x & 1) * (kSrTCX + 1) + (x >> 1)]; };
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int tile = lb % tiles, run = lb / tiles;
  const int n0 = run * RL;
  double ssq = 0.0;
  if (n0 < p.N) {
    const int n1 = min(n0 + RL, p.N);
    const Consts<M, T> c(p);
    const T dg = T(2) * c.cx + T(2) * c.cy;
    const int nx = p.nx, ny = p.ny, P = nx * ny, Pc = ncx * ncy;
    const int X0 = (tile % tiles_x) * kSrTCX, Y0 = (tile / tiles_x) * kSrTCY;
    const int tx = threadIdx.x % kSrTCX, ty = threadIdx.x / kSrTCX;
    const int X = X0 + tx, Y = Y0 + ty;
    const Blk<2> b(Y * (nx >> 1) + X, nx, ny);
    T* __restrict__ out = static_cast<T*>(a.out);
    // ring point of this thread
    const bool ring = threadIdx.x < kSrRing;
    const bool rhalo = threadIdx.x < kSrRHalo;
    int rlx = 0, rly = 0;
    if (ring) sr_ring_point(threadIdx.x, rlx, rly);
    int rfx = 2 * X0 + rlx, rfy = 2 * Y0 + rly;
    if (rfx < 0) rfx += nx;
    if (rfx >= nx) rfx -= nx;
    if (rfy < 0) rfy += ny;
    if (rfy >= ny) rfy -= ny;
    const int rq = rfy * nx + rfx;
    const Nbr rn = neighbours(rfx, rfy, nx, ny, 0);
    // coupling values entering the run
    T prev[4], dprev[4];
    run_prev<M, T, 2>(c, a, n0, P, nx, b, prev);
#pragma unroll
    for (int k = 0; k < 4; ++k) dprev[k] = T(0);
    T rprev = T(0), rdprev = T(0);
    if (ring) {
      if (n0 == 0) {
        if (a.u0) rprev = (T)a.u0[rq];
      } else if (a.U) {
        const size_t bb = (size_t)(n0 - 1) * M * P;
#pragma unroll
        for (int j = 0; j < M; ++j) rprev += c.cout[j] * a.U[bb + (size_t)j * P + rq];
      }
    }
    const int qc = Y * ncx + X;
    T zdprev = T(0);
    // the block's own rows of the next slab are loaded at the end of the
    // current slab's sweep, so their memory latency overlaps its residual
    // and restriction phases
    T own[M][2][2];
    if (a.U) load_rows<M, T, 2>(a.U, (size_t)n0 * M * P, P, b, own);
    for (int n = n0; n < n1; ++n) {
      const size_t base = (size_t)n * M * P;
      // (1) the sweep: own block, then the ring point
      T u[4][M], lap[4][M], fv[4][M], r[4][M], d[4][M], o[2][M];
      // the ring point's values are loaded with the block's (every thread
      // loads a valid point: without a ring point, the tile's corner), so a
      // slab step waits for one round of loads
      T ru[M], rl[M], rfv[M], rcv[M];
      if (a.U) {
        blk_from_rows<M, T, 2, true>(a.U, base, P, b, c.cx, c.cy, own, u, lap);
        load_point<M, T>(a.U, base, P, rq, rn, true, c.cx, c.cy, ru, rl);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) u[k][m] = lap[k][m] = T(0);
#pragma unroll
        for (int m = 0; m < M; ++m) ru[m] = rl[m] = T(0);
      }
#pragma unroll
      for (int i = 0; i < M; ++i) {
        rcv[i] = REACT == REACT_COEF ? a.coef[base + (size_t)i * P + rq] : T(0);
        rfv[i] = HASF ? a.f[base + (size_t)i * P + rq] : T(0);
      }
      T cv[4][M];
      if (REACT == REACT_COEF) load_own<M, T, 2>(a.coef, base, P, nx, b, cv);
      if (HASF) {
        load_own<M, T, 2>(a.f, base, P, nx, b, fv);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) fv[k][m] = T(0);
      }
      T* __restrict__ orow0 = out + base;
      // a smoother chunk starts at n: no coupling in the sweep; inside the
      // run the residual of U' takes the chunk-start term with cout . d_{n-1}
      const bool cstart = (n % chunk) == 0;
      const bool cterm = cstart && n > n0;
      T zp[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        zp[k] = dprev[k];
        resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], r[k]);
        if (a.part) ssq_add<M, T>(p, r[k], ssq);
        T x[M];
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] = cstart ? r[k][i] : r[k][i] + c.cin[i] * dprev[k];
        // the point block solve (with the point's reaction coefficient for REACT_COEF)
        const T nd = point_correction<M, T, REACT>(c, dg, cv[k], x, d[k]);
        T np = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          o[k & 1][i] = u[k][i] + c.omega * d[k][i];
          np += c.cout[i] * u[k][i];
        }
        prev[k] = np;
        dprev[k] = nd;
        const int lx = 2 * tx + (k & 1), ly = 2 * ty + (k >> 1);
#pragma unroll
        for (int i = 0; i < M; ++i) dt(i, ly, lx) = d[k][i];
        if (k & 1) {
          // the row pair (2X, 2X + 1) of fine row 2Y + k / 2 is complete
          const int q0 = b.q(k - 1, nx);
#pragma unroll
          for (int i = 0; i < M; ++i) {
            typedef T v2 __attribute__((ext_vector_type(2)));
            v2 v;
            v.x = o[0][i];
            v.y = o[1][i];
            __builtin_nontemporal_store(v, reinterpret_cast<v2*>(orow0 + (size_t)i * P + q0));
          }
        }
      }
      T hr[M];
      const T rzp = rdprev;
      resid_vals<M, T, REACT>(c, ru, rl, rfv, rcv, rprev, hr);
      if (ring) {
        T x[M], rd[M];
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] = cstart ? hr[i] : hr[i] + c.cin[i] * rdprev;
        const T nd = point_correction<M, T, REACT>(c, dg, rcv, x, rd);
        T np = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          dt(i, rly, rlx) = rd[i];
          np += c.cout[i] * ru[i];
        }
        rprev = np;
        rdprev = nd;
      }
      if (a.U && n + 1 < n1) load_rows<M, T, 2>(a.U, base + (size_t)M * P, P, b, own);
      __syncthreads();
      // (2) residuals of U': (1 - omega) r + omega db (cx (d_W + d_E) + cy (d_S + d_N))
      const T om = c.omega, om1 = T(1) - c.omega;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i0 = k & 1, j0 = k >> 1;
        const int lx = 2 * tx + i0, ly = 2 * ty + j0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const T dw = i0 == 1 ? d[k - 1][m] : dt(m, ly, lx - 1);
          const T de = i0 == 0 ? d[k + 1][m] : dt(m, ly, lx + 1);
          const T ds = j0 == 1 ? d[k - 2][m] : dt(m, ly - 1, lx);
          const T dn = j0 == 0 ? d[k + 2][m] : dt(m, ly + 1, lx);
          T v = om1 * r[k][m] + om * c.db[m] * (c.cx * (dw + de) + c.cy * (ds + dn));
          if (cterm) v += om * c.cin[m] * zp[k];
          rt(m, ly + 1, lx + 1) = v;
        }
      }
      if (rhalo) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const T dw = dt(m, rly, rlx - 1), de = dt(m, rly, rlx + 1);
          const T ds = dt(m, rly - 1, rlx), dn = dt(m, rly + 1, rlx);
          T v = om1 * hr[m] + om * c.db[m] * (c.cx * (dw + de) + c.cy * (ds + dn));
          if (cterm) v += om * c.cin[m] * rzp;
          rt(m, rly + 1, rlx + 1) = v;
        }
      }
      __syncthreads();
      // (3) full weighting to the coarse point, coarse first sweep
      T rc[M];
      const int cx0 = 2 * tx, cy0 = 2 * ty;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T s0 = T(0.25) * rt(i, cy0, cx0) + T(0.5) * rt(i, cy0, cx0 + 1) + T(0.25) * rt(i, cy0, cx0 + 2);
        const T s1 = T(0.25) * rt(i, cy0 + 1, cx0) + T(0.5) * rt(i, cy0 + 1, cx0 + 1) +
                     T(0.25) * rt(i, cy0 + 1, cx0 + 2);
        const T s2 = T(0.25) * rt(i, cy0 + 2, cx0) + T(0.5) * rt(i, cy0 + 2, cx0 + 1) +
                     T(0.25) * rt(i, cy0 + 2, cx0 + 2);
        rc[i] = T(0.25) * s0 + T(0.5) * s1 + T(0.25) * s2;
      }
      const size_t cb = (size_t)n * M * Pc;
#pragma unroll
      for (int i = 0; i < M; ++i) __builtin_nontemporal_store(rc[i], fc + cb + (size_t)i * Pc + qc);
      if (ZS) {
        const Consts<M, T> k(pc);
        const T dgc = T(2) * k.cx + T(2) * k.cy;
        T rr[M], cvv[M], dd[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
          rr[i] = rc[i] + ((n % cs) != 0 ? k.cin[i] * zdprev : T(0));
          cvv[i] = REACT == REACT_COEF ? coefc[cb + (size_t)i * Pc + qc] : T(0);
        }
        zdprev = point_correction<M, T, REACT>(k, dgc, cvv, rr, dd);
#pragma unroll
        for (int i = 0; i < M; ++i) __builtin_nontemporal_store(k.omega * dd[i], uc + cb + (size_t)i * Pc + qc);
      }
    }
    // cout . d of the run's last slab, for the next run's first slab
    if (n1 < p.N) {
      T* z = zbuf + (size_t)run * P;
#pragma unroll
      for (int k = 0; k < 4; ++k) z[b.q(k, nx)] = dprev[k];
    }
  }
  if (a.part) {
    const double tt = block_sum(ssq);
    if (threadIdx.x == 0) a.part[lb] = tt;
  }
}

// The first slab J of every run but the first: f_c[J] += omega cin R z with
// z = cout . d of slab J - 1 (full weighting, periodic), and with ZS the
// coarse sweep's response along the coarse chunk that J starts.
template <int M, typename T, int REACT, bool ZS>
__global__ __launch_bounds__(kBlock) void k_sr_fixup(const OpParams p, int ncx, int ncy, int RL, int nbound,
                                                     T* __restrict__ fc, const OpParams pc, T* __restrict__ uc,
                                                     const T* __restrict__ coefc, int cs,
                                                     const T* __restrict__ zbuf) {
  const int Pc = ncx * ncy;
  const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= (long long)Pc * nbound) return;
  const int bd = (int)(idx / Pc), qc = (int)(idx - (long long)bd * Pc);
  const int X = qc % ncx, Y = qc / ncx;
  const int nx = p.nx, ny = p.ny;
  const int J = (bd + 1) * RL;
  const T* z = zbuf + (size_t)bd * nx * ny;
  const int x0 = 2 * X, y0 = 2 * Y;
  const int xm = x0 > 0 ? x0 - 1 : nx - 1, xp = x0 + 1;
  const int ym = y0 > 0 ? y0 - 1 : ny - 1, yp = y0 + 1;
  auto row = [&](int y) {
    return T(0.25) * z[y * nx + xm] + T(0.5) * z[y * nx + x0] + T(0.25) * z[y * nx + xp];
  };
  const T s = (T)p.omega * (T(0.25) * row(ym) + T(0.5) * row(y0) + T(0.25) * row(yp));
  const Consts<M, T> c(p);
  const size_t cb = (size_t)J * M * Pc;
#pragma unroll
  for (int i = 0; i < M; ++i) fc[cb + (size_t)i * Pc + qc] += c.cin[i] * s;
  if (ZS) {
    const Consts<M, T> k(pc);
    const T dgc = T(2) * k.cx + T(2) * k.cy;
    const int nj = min(cs, p.N - J);
    // the chunk's values are read before the recurrence (at most kSrMaxCs slabs)
    T ucv[kSrMaxCs][M];
#pragma unroll
    for (int jj = 0; jj < kSrMaxCs; ++jj)
#pragma unroll
      for (int i = 0; i < M; ++i) ucv[jj][i] = jj < nj ? uc[(size_t)(J + jj) * M * Pc + (size_t)i * Pc + qc] : T(0);
    T zd = T(0);
#pragma unroll
    for (int jj = 0; jj < kSrMaxCs; ++jj) {
      if (jj < nj) {
        T rr[M], cvv[M], dd[M];
        const size_t cj = (size_t)(J + jj) * M * Pc;
#pragma unroll
        for (int i = 0; i < M; ++i) {
          rr[i] = jj == 0 ? c.cin[i] * s : k.cin[i] * zd;
          cvv[i] = REACT == REACT_COEF ? coefc[cj + (size_t)i * Pc + qc] : T(0);
        }
        zd = point_correction<M, T, REACT>(k, dgc, cvv, rr, dd);
#pragma unroll
        for (int i = 0; i < M; ++i) uc[cj + (size_t)i * Pc + qc] = ucv[jj][i] + k.omega * dd[i];
      }
    }
  }
}

}  // namespace

bool smooth_restrict_ok(const OpParams& p, int react, int ncx, int ncy, int Nc, int chunk, int cs) {
  return p.bc == 0 && p.ny > 1 && (react == REACT_CONST || react == REACT_COEF) && p.M >= 1 && p.M <= 4 && p.nx % kSrFX == 0 &&
         p.ny % kSrFY == 0 && ncx * 2 == p.nx && ncy * 2 == p.ny && Nc == p.N && chunk >= 1 && cs >= 1 &&
         cs <= kSrMaxCs && chunk % cs == 0;
}

// Slabs per workgroup: whole smoother chunks, doubled while the launch
// still has two workgroups per CU (fewer run boundaries for k_sr_fixup).
static int sr_run_len(const OpParams& p, int chunk) {
  const long long tiles = (long long)(p.nx / kSrFX) * (p.ny / kSrFY);
  int rl = chunk;
  while (rl < p.N && tiles * ((p.N + 2 * rl - 1) / (2 * rl)) >= 512) rl *= 2;
  return rl;
}

int smooth_restrict_blocks(const OpParams& p, int chunk) {
  const int rl = sr_run_len(p, chunk);
  return (p.nx / kSrFX) * (p.ny / kSrFY) * ((p.N + rl - 1) / rl);
}

size_t smooth_restrict_zbuf(const OpParams& p, int chunk) {
  const int rl = sr_run_len(p, chunk);
  const int runs = (p.N + rl - 1) / rl;
  return runs > 1 ? static_cast<size_t>(runs - 1) * p.nx * p.ny : 0;
}

template <typename T>
hipError_t launch_smooth_restrict(const OpParams& p, int react, const SweepPtrs<T>& a, int ncx, int ncy, T* fc,
                                  int chunk, const OpParams* pc, T* uc, const T* coefc, int cs, T* zbuf,
                                  hipStream_t s) {
  if (!smooth_restrict_ok(p, react, ncx, ncy, p.N, chunk, cs) || !a.out || !fc) return hipErrorInvalidValue;
  const bool coef = react == REACT_COEF;
  const bool zs = uc != nullptr && pc != nullptr;
  if (coef && (!a.coef || (zs && !coefc))) return hipErrorInvalidValue;
  const OpParams& pcc = zs ? *pc : p;
  const int tiles_x = ncx / kSrTCX;
  const int tiles = tiles_x * (ncy / kSrTCY);
  const int rl = sr_run_len(p, chunk);
  const int nb = smooth_restrict_blocks(p, chunk);
  const int runs = (p.N + rl - 1) / rl;
  if (runs > 1 && !zbuf) return hipErrorInvalidValue;
  const long long work = (long long)ncx * ncy * (runs - 1);
  const int fb = (int)((work + kBlock - 1) / kBlock);
#define LK(MM, RE, ZZ, FF)                                                                                     \
  hipLaunchKernelGGL((k_smooth_restrict<MM, T, RE, ZZ, FF>), dim3(nb), dim3(kBlock), 0, s, p, a, ncx, ncy, fc, rl, \
                     chunk, tiles_x, tiles, nb, pcc, uc, coefc, cs, zbuf)
#define LF(MM, RE, ZZ)                                                                                         \
  hipLaunchKernelGGL((k_sr_fixup<MM, T, RE, ZZ>), dim3(fb), dim3(kBlock), 0, s, p, ncx, ncy, rl, runs - 1, fc, \
                     pcc, uc, coefc, cs, zbuf)
#define LR(MM, RE)                                                                                             \
  if (zs) { if (a.f) LK(MM, RE, true, true); else LK(MM, RE, true, false); }                                   \
  else { if (a.f) LK(MM, RE, false, true); else LK(MM, RE, false, false); }                                    \
  if (runs > 1) { if (zs) LF(MM, RE, true); else LF(MM, RE, false); }
  // FP64 with a reaction coefficient needs over 240 registers (one or two
  // waves per SIMD): the separate kernels serve it
  if constexpr (sizeof(T) == 8) {
    if (coef) return hipErrorNotSupported;
  }
#define L(MM)                                             \
  if constexpr (sizeof(T) == 8) { LR(MM, REACT_CONST) }   \
  else { if (coef) { LR(MM, REACT_COEF) } else { LR(MM, REACT_CONST) } }
  switch (p.M) {
    case 1: L(1); break;
    case 2: L(2); break;
    case 3: L(3); break;
    case 4: L(4); break;
    default: return hipErrorInvalidValue;
  }
#undef L
#undef LR
#undef LF
#undef LK
  return hipGetLastError();
}

template hipError_t launch_smooth_restrict<double>(const OpParams&, int, const SweepPtrs<double>&, int, int, double*,
                                                   int, const OpParams*, double*, const double*, int, double*,
                                                   hipStream_t);
template hipError_t launch_smooth_restrict<float>(const OpParams&, int, const SweepPtrs<float>&, int, int, float*, int,
                                                  const OpParams*, float*, const float*, int, float*, hipStream_t);

}  // namespace stmg
