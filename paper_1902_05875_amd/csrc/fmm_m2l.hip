// M2L on the matrix cores (gfx950 MFMA 16x16x4, FP64 or FP32).
//
// Sec. 3.1 / Eq. tesourceboxtotargetbox: beta_k = sum_k' alpha_k' D^k D'^k' F / (k! k'!).
// With box-scaled moments and locals and G_g = h^{|g|} D^g F (the derivative
// table of the key) this becomes the Hankel contraction
//     b_k = sum_{k'} G_{k+k'} a_{k'},   a_{k'} = s (-1)^{|k'|} alpha^_{k'} / k'!,
//     beta^_k = b_k / k!,
// with s = (-1)^{k3'} for the Sigma family (whose kernel depends on z + z',
// so that source derivatives in z enter with a plus sign) and s = 1 otherwise.
// Both a and b are used in the Helmholtz-reduced form (k1 <= 1, (p+1)^2
// entries; see k_reduce / k_expand), so the operator is (p+1)^2 x (p+1)^2 and
// only table entries with g1 <= 2 are read.
//
// Work decomposition: a workgroup owns a tile of 16 target boxes that share
// z index and the parity of x and y (so all 16 have the same 6x6x6 window of
// candidate source offsets and the same table keys); it loops over the window
// and, per offset, stages the key's compact table (C(2p+3,3) complex values)
// and the 16 source moment vectors in LDS.  MFMA rows are output indices k,
// columns the 16 targets, K the source index k'; the A operand G_{k+k'} is
// gathered from the compact table in LDS.  Four waves split the row blocks.
#include <hip/hip_runtime.h>

#include <utility>

#include "fmm_kernels.hpp"
#include "kernels.hpp"

namespace tefmm {

template <typename T>
struct M2LTypes;
template <>
struct M2LTypes<double> {
  typedef double2 T2;
  typedef d4 acc;
  __device__ static acc mfma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static const T2* tableF(const M2LLevel& L) { return L.Tfd; }
  __device__ static const T2* tableS(const M2LLevel& L) { return L.TS; }
  __device__ static T2 cvt(double2 v) { return v; }
  // FP64 16x16x4 result: register i of lane l holds row (l >> 4) + 4 i, column l & 15
  __device__ static int row(int lane_hi, int i) { return lane_hi + 4 * i; }
};
template <>
struct M2LTypes<float> {
  typedef float2 T2;
  typedef f4 acc;
  __device__ static acc mfma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static const T2* tableF(const M2LLevel& L) { return L.Tfd32; }
  __device__ static const T2* tableS(const M2LLevel& L) { return L.TS32; }
  __device__ static T2 cvt(double2 v) { return make_float2((float)v.x, (float)v.y); }
  // FP32 16x16x4 result: register i of lane l holds row 4 (l >> 4) + i, column l & 15
  __device__ static int row(int lane_hi, int i) { return 4 * lane_hi + i; }
};

// LDS layout of a key's table: G_{k+k'} sits at ((g1 P2 + m) P2 + g3) with
// g1 = k1 + k1', m = (k2 + k3) + (k2' + k3'), g3 = k3 + k3', P2 = 2p + 1, so
// the address splits into a row part and a column part:
//   row(k) = (k1 P2 + k2 + k3) P2 + k3,  col(k') = (k1' P2 + k2' + k3') P2 + k3'.

// Valid-target bit mask of a tile for a source offset (dx, dy): target n sits
// at x index px + 2 (4 X0 + (n & 3)), y index py + 2 (4 NCB Y0 + (n >> 2)).
template <int NCB>
__device__ __forceinline__ unsigned tile_mask(int N, int px, int py, int X0, int Y0, int dx, int dy) {
  unsigned xm = 0, m = 0;
#pragma unroll
  for (int xi = 0; xi < 4; ++xi) {
    const int ix = px + 2 * (4 * X0 + xi);
    xm |= (ix < N && ix + dx >= 0 && ix + dx < N) ? (1u << xi) : 0u;
  }
#pragma unroll
  for (int yi = 0; yi < 4 * NCB; ++yi) {
    const int iy = py + 2 * (4 * NCB * Y0 + yi);
    m |= (iy < N && iy + dy >= 0 && iy + dy < N) ? (xm << (4 * yi)) : 0u;
  }
  return m;
}

// EX: every wave has TW tiles (4 TW row-block x column-block tiles in all), no test.
// KS = 1 or 2: 4 (TW - 1) + KS tiles; each wave has TW - 1 tiles of its own, and the
// last KS tiles are split along the contraction (KS = 1: the tile's K blocks in four
// quarters, one per wave; KS = 2: each of the two tiles in two halves, waves 0 and 1
// on the first, 2 and 3 on the second), so that every wave does the same number of
// MFMAs; the waves' partial sums of a split tile are added in wave order in LDS.
template <typename T, int TW, int NCB, bool EX, int KS>
__global__ __launch_bounds__(256) void k_m2l(M2LArgs a) {
  typedef M2LTypes<T> Ty;
  typedef typename Ty::T2 T2;
  typedef typename Ty::acc AC;
  constexpr int NT = 16 * NCB;  // target boxes per workgroup
  extern __shared__ double lds_m2l[];
  const int P2 = a.P2;
  const int padG = 3 * P2 * P2;
  T2* sG = (T2*)lds_m2l;
  T2* sA = sG + padG + 1;  // sG[padG]: a zero read by lanes with no table entry
  int* sCol = (int*)(sA + NT * a.nRsP);    // [4 nKB]: column offset | k3' parity << 20 | valid << 21

  // Block -> (level, tile).  The widest level's tiles come first (they hold the most
  // offsets, so the coarse levels' shorter workgroups are dealt out last), remapped so
  // that consecutive tiles (same z slab) stay on one XCD; the coarse levels keep the
  // hardware's round-robin over the XCDs.
  int li = 0, tile = 0;
  const int widest = a.nlev - 1;
  const int nwide = a.tile_start[widest + 1] - a.tile_start[widest];  // a multiple of 8
  if ((int)blockIdx.x >= nwide) {
    const int bc = blockIdx.x - nwide;
    while (bc >= a.tile_start[li + 1]) ++li;
    tile = bc - a.tile_start[li];
  } else {
    li = widest;
    const int b = blockIdx.x;
    const int nt = a.lev[li].ntiles;
    const int per = (nt + 7) / 8;
    tile = (b % 8) * per + b / 8;
    if (tile >= nt) return;
  }
  const M2LLevel& L = a.lev[li];
  const int r = blockIdx.y, split = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  int t = tile;
  const int X0 = t % L.tiles_x;
  t /= L.tiles_x;
  const int Y0 = t % L.tiles_y;
  t /= L.tiles_y;
  const int px = t & 1, py = (t >> 1) & 1, iz = t >> 2;
  const int N = L.n, pz = iz & 1;
  int ocount = 0;  // offsets with work so far; this workgroup takes those with ocount % nsplit == split
  // target n: ix = px + 2 (4 X0 + (n & 3)), iy = py + 2 (4 NCB Y0 + (n >> 2))
  unsigned tmask = 0;
  for (int n = 0; n < NT; ++n) {
    const int ix = px + 2 * (4 * X0 + (n & 3)), iy = py + 2 * (4 * NCB * Y0 + (n >> 2));
    if (ix < N && iy < N) tmask |= 1u << n;
  }
  // Occupancy of the boxes the tile can reach (x from px + 8 X0 - 3, y from
  // py + 8 NCB Y0 - 3, z from iz - 3: the offsets reach three boxes either way).
  // Empty boxes have zero moments and no particle reads their locals, so empty
  // targets keep zero locals and empty sources are skipped: the occupied boxes'
  // locals are the same sums.
  constexpr int WX = 13, WY = 8 * NCB + 5, WZ = 7;
  unsigned char* sOcc = (unsigned char*)(sCol + 4 * a.nKB);
  unsigned tocc = tmask;
  if (L.occ) {
    const int x0 = px + 8 * X0 - 3, y0 = py + 8 * NCB * Y0 - 3, z0 = iz - 3;
    for (int e = tid; e < WX * WY * WZ; e += 256) {
      const int wx = e / (WY * WZ), wy = (e / WZ) % WY, wz = e % WZ;
      const int x = x0 + wx, y = y0 + wy, z = z0 + wz;
      sOcc[e] = (x >= 0 && y >= 0 && z >= 0 && x < N && y < N && z < N) ? L.occ[((int64_t)x * N + y) * N + z] : 0;
    }
    __syncthreads();
    unsigned m = 0;
    for (int n = 0; n < NT; ++n)
      if (sOcc[((3 + 2 * (n & 3)) * WY + 3 + 2 * (n >> 2)) * WZ + 3]) m |= 1u << n;
    tocc = __builtin_amdgcn_readfirstlane(m) & tmask;
  }

  // reduced moments: FP32 copies in the mixed mode
  const double2* alpha = L.a ? L.a + (int64_t)r * L.rhs_stride : nullptr;
  const float2* alpha32 = L.a32 ? L.a32 + (int64_t)r * L.rhs_stride : nullptr;
  for (int e = tid; e < NT * a.nRsP; e += 256) {
    sA[e].x = 0;
    sA[e].y = 0;
  }
  for (int e = tid; e <= padG; e += 256) {
    sG[e].x = 0;
    sG[e].y = 0;
  }
  for (int e = tid; e < 4 * a.nKB; e += 256) {
    int v = 0;
    if (e < a.nR) {
      const int pk = a.rmi[e];
      const int k1 = pk & 255, k2 = (pk >> 8) & 255, k3 = pk >> 16;
      v = ((k1 * P2 + k2 + k3) * P2 + k3) | ((k3 & 1) << 20) | (1 << 21);
    }
    sCol[e] = v;
  }

  // this wave's (row block, column block) tiles, round robin over the 4 waves
  const int col = lane & 15, krow = lane >> 4;
  const int ntile = a.nRB * NCB;
  int rowo[TW], tcb[TW];
#pragma unroll
  for (int j = 0; j < TW; ++j) {
    const int id = (KS && j == TW - 1) ? 4 * (TW - 1) + (KS == 1 ? 0 : (w >> 1)) : w + 4 * j;
    const int rb = id % a.nRB, cb = id / a.nRB;
    const int k = 16 * rb + col;
    // rows past nR (and missing tiles) gather entry 0: finite, and dropped by the epilogue
    rowo[j] = 0, tcb[j] = cb;
    if (id < ntile && k < a.nR) {
      const int pk = a.rmi[k];
      const int k1 = pk & 255, k2 = (pk >> 8) & 255, k3 = pk >> 16;
      rowo[j] = (k1 * P2 + k2 + k3) * P2 + k3;
    }
  }
  // K blocks [kq0, kq1) of the split tile taken by this wave (wave-uniform)
  const int kq0 = KS == 1 ? (w * a.nKB) / 4 : KS == 2 ? ((w & 1) * a.nKB) / 2 : 0;
  const int kq1 = KS == 1 ? ((w + 1) * a.nKB) / 4 : KS == 2 ? (((w & 1) + 1) * a.nKB) / 2 : 0;
  // B operand offset of each tile: column block tcb, target col
  int boff[TW];
#pragma unroll
  for (int j = 0; j < TW; ++j) boff[j] = (16 * tcb[j] + col) * a.nRsP;
  // Complex products by three real products (Gauss): with G = g + i h and a = c + i d,
  // s1 = (g + h) c, s2 = g (d - c), s3 = h (c + d), Re G a = s1 - s3, Im G a = s1 + s2;
  // the three sums are formed in registers from the staged values and combined in FP64
  // at the end
  constexpr bool F32 = sizeof(T) == 4;
  AC acc1[TW], acc2[TW], acc3[TW];
  const bool last_ok = w + 4 * (TW - 1) < ntile;  // wave-uniform
#pragma unroll
  for (int j = 0; j < TW; ++j) {
    acc1[j] = AC{0, 0, 0, 0};
    acc2[j] = AC{0, 0, 0, 0};
    acc3[j] = AC{0, 0, 0, 0};
  }

  // staging constants: thread's first element, the per-step advance, and the
  // moment address of target n at offset (0, 0, 0):
  //   ((ix N + iy) N + iz) nR with ix = px + 2 (4 X0 + (n & 3)), iy = py + 2 (4 NCB Y0 + (n >> 2))
  // the moments of a phase: k' in [4 kpb ph, 4 kpb (ph + 1)), element e = (n, k' - base)
  const int Lp = 4 * a.kpb;
  const int n0 = tid / Lp, kk0 = tid - n0 * Lp;
  const int step_q = 256 / Lp, step_r = 256 - step_q * Lp;
  int tbase[4];
#pragma unroll
  for (int xi = 0; xi < 4; ++xi)
    tbase[xi] = (((px + 2 * (4 * X0 + xi)) * N + (py + 8 * NCB * Y0)) * N + iz) * a.nR;
  const int tbase_y = 2 * N * a.nR;
  // Staging by runs: with at most two phases, E = NT Lp / 256 even and dividing Lp, and
  // nR even, each thread stages E consecutive entries of one target (loaded two at a
  // time), with the validity and the Sigma sign of each entry fixed per thread and phase.
  const int E = (NT * Lp) / 256;
  const bool runs = a.kph <= 2 && (NT * Lp) % 256 == 0 && E % 2 == 0 && E <= 8 && Lp % E == 0 && a.nR % 2 == 0;
  const int rn = runs ? (tid * E) / Lp : 0, rk = runs ? (tid * E) % Lp : 0;
  unsigned rvalid[2] = {0u, 0u}, rsign[2] = {0u, 0u};
  __syncthreads();  // sCol complete
  if (runs)
    for (int ph = 0; ph < a.kph; ++ph)
      for (int i = 0; i < E; ++i) {
        const int kk = Lp * ph + rk + i;
        if (kk < a.nR) rvalid[ph] |= 1u << i, rsign[ph] |= (unsigned)((sCol[kk] >> 20) & 1) << i;
      }
  const int npass = tocc ? 2 : 0;  // no occupied target: zero locals
  for (int pass = 0; pass < npass; ++pass) {
    const T2* table = pass ? (const T2*)Ty::tableS(L) : (const T2*)Ty::tableF(L);
    if (!table) continue;
    const bool mirror = pass == 1;
    const bool near_ok = pass ? L.near_s : L.near_fd;
    for (int oz = 0; oz < 6; ++oz) {
      const int dz = oz - 2 - pz;
      if (iz + dz < 0 || iz + dz >= N) continue;
      for (int oy = 0; oy < 6; ++oy) {
        const int dy = oy - 2 - py;
        for (int ox = 0; ox < 6; ++ox) {
          const int dx = ox - 2 - px;
          const bool nearb = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
          if (nearb && !(L.leaf && near_ok)) continue;
          unsigned smask = tile_mask<NCB>(N, px, py, X0, Y0, dx, dy);
          if (L.occ) {  // lane n < NT tests target n's source box; the same mask in every wave
            const int l = lane < NT ? lane : 0;
            const bool o = lane < NT && sOcc[((3 + 2 * (l & 3) + dx) * WY + 3 + 2 * (l >> 2) + dy) * WZ + 3 + dz];
            smask &= (unsigned)__ballot(o) & tocc;
          }
          if (!smask) continue;
          if ((ocount++) % a.nsplit != split) continue;
          const int key = pass ? ((dx + 3) * 7 + (dy + 3)) * (2 * N - 1) + (2 * iz + dz)
                               : ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3);
          const int delta = ((dx * N + dy) * N + dz) * a.nR;
          for (int ph = 0; ph < a.kph; ++ph) {
            const int kbase = Lp * ph;
            __syncthreads();
            if (ph == 0) {
              const T2* g = table + (int64_t)key * a.nG;
              for (int e = tid; e < a.nG; e += 256) sG[a.gpad[e]] = g[e];
            }
            if (runs) {
              const bool on = (smask >> rn) & 1;
              const int64_t at = tbase[rn & 3] + tbase_y * (rn >> 2) + kbase + rk + delta;
              const unsigned neg = mirror ? rsign[ph] : 0u;
              T2* dst = sA + rn * a.nRsP + rk;
#pragma unroll
              for (int i = 0; i < 8; i += 2) {
                if (i >= E) break;
                T2 v0, v1;
                v0.x = 0, v0.y = 0, v1.x = 0, v1.y = 0;
                if (on && ((rvalid[ph] >> i) & 1)) {
                  if (F32) {
                    const float4 q = *(const float4*)(alpha32 + at + i);
                    v0.x = (T)q.x, v0.y = (T)q.y, v1.x = (T)q.z, v1.y = (T)q.w;
                  } else {
                    const double2 q0 = alpha[at + i], q1 = alpha[at + i + 1];
                    v0 = Ty::cvt(q0), v1 = Ty::cvt(q1);
                  }
                  if ((neg >> i) & 1) v0.x = -v0.x, v0.y = -v0.y;
                  if ((neg >> (i + 1)) & 1) v1.x = -v1.x, v1.y = -v1.y;
                }
                dst[i] = v0, dst[i + 1] = v1;
              }
            } else {
              // element e = tid + 256 i of the NT x Lp moment block: target n, index kk
              // (advanced by 256 = q Lp + rem per step, without a division per element)
              int n = n0, kl = kk0;
              for (int e = tid; e < NT * Lp; e += 256) {
                const int kk = kbase + kl;
                T2 v;
                v.x = 0;
                v.y = 0;
                if (kk < a.nR && ((smask >> n) & 1)) {
                  const double s = (mirror && ((sCol[kk] >> 20) & 1)) ? -1.0 : 1.0;
                  const int64_t at = tbase[n & 3] + tbase_y * (n >> 2) + kk + delta;
                  if (sizeof(T) == 4) {
                    const float2 av = alpha32[at];
                    v.x = (T)(av.x * (float)s), v.y = (T)(av.y * (float)s);
                  } else {
                    const double2 av = alpha[at];
                    v = Ty::cvt(make_double2(av.x * s, av.y * s));
                  }
                }
                sA[n * a.nRsP + kl] = v;
                n += step_q, kl += step_r;
                if (kl >= Lp) kl -= Lp, ++n;
              }
            }
            __syncthreads();
            const int kb0 = a.kpb * ph, kb1 = min(a.nKB, a.kpb * (ph + 1));
            // operands of block kb: B from the staged moments, A gathered from the table
            // (sG[padG] = 0 where the lane has no entry); those of kb + 1 are loaded while
            // the MFMAs of kb run
            // operands of block kb: B from the staged moments (per tile when the wave has
            // at most two tiles, else the two column blocks and a select), A gathered from the
            // table; those of the next block are loaded while the MFMAs of this one run (two
            // register sets used in turn)
            constexpr bool BT = TW <= 2;
            auto load = [&](int kb, T2 (&bb)[TW], T2 (&g)[TW]) {
              const int kp = 4 * kb + krow;
              // column offset; 0 past nR, where the staged moments are zero
              const int co = sCol[kp] & 0xFFFFF;
              if (BT) {
#pragma unroll
                for (int j = 0; j < TW; ++j) bb[j] = sA[boff[j] + kp - kbase];
              } else {
                bb[0] = sA[col * a.nRsP + kp - kbase];
                if (NCB == 2) bb[1] = sA[(16 + col) * a.nRsP + kp - kbase];
              }
#pragma unroll
              for (int j = 0; j < TW; ++j) g[j] = sG[rowo[j] + co];
            };
            auto mma = [&](const T2 (&bb)[TW], const T2 (&g)[TW], int kb) {
              // independent MFMAs between the two updates of each accumulator; only the
              // wave's last tile can be missing (ntile > 4 (TW - 1)) or split (its K
              // blocks outside [kq0, kq1) are another wave's), a uniform test
              const bool lon = KS ? (kb >= kq0 && kb < kq1) : last_ok;
              // B operand of tile j: its own load (BT), else column block tcb[j] (always 0
              // with one column block)
              constexpr int NB = BT ? TW : NCB;
              auto bsel = [&](const T (&v)[NB], int j) { return BT ? v[j] : (NCB == 2 && tcb[j] ? v[NB - 1] : v[0]); };
              T bc[NB], dmc[NB], cpd[NB];
#pragma unroll
              for (int u = 0; u < NB; ++u) bc[u] = bb[u].x, dmc[u] = bb[u].y - bb[u].x, cpd[u] = bb[u].x + bb[u].y;
#pragma unroll
              for (int j = 0; j < TW; ++j)
                if (EX || j < TW - 1 || lon) acc1[j] = Ty::mfma(g[j].x + g[j].y, bsel(bc, j), acc1[j]);
#pragma unroll
              for (int j = 0; j < TW; ++j)
                if (EX || j < TW - 1 || lon) acc2[j] = Ty::mfma(g[j].x, bsel(dmc, j), acc2[j]);
#pragma unroll
              for (int j = 0; j < TW; ++j)
                if (EX || j < TW - 1 || lon) acc3[j] = Ty::mfma(g[j].y, bsel(cpd, j), acc3[j]);
            };
            T2 b1[TW], g1[TW], b2[TW], g2[TW];
            if (kb0 < kb1) load(kb0, b1, g1);
            for (int kb = kb0; kb < kb1; kb += 2) {
              if (kb + 1 < kb1) load(kb + 1, b2, g2);
              mma(b1, g1, kb);
              if (kb + 1 >= kb1) break;
              if (kb + 2 < kb1) load(kb + 2, b1, g1);
              mma(b2, g2, kb + 1);
            }
          }
        }
      }
    }
  }
  // epilogue: result rows per the precision's MFMA layout, columns = targets
  double2* beta = L.b + (int64_t)split * L.split_stride + (int64_t)r * L.rhs_stride;
#pragma unroll
  for (int j = 0; j < (KS ? TW - 1 : TW); ++j) {
    const int id = w + 4 * j;
    if (id >= ntile) continue;
    const int rb = id % a.nRB, cb = id / a.nRB;
    const int n = 16 * cb + col;
    if (!((tmask >> n) & 1)) continue;
    const int ix = px + 2 * (4 * X0 + (n & 3)), iy = py + 2 * (4 * NCB * Y0 + (n >> 2));
    const int64_t tb = ((int64_t)ix * N + iy) * N + iz;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 16 * rb + Ty::row(krow, i);
      if (k < a.nR) {
        const double s1 = (double)acc1[j][i];
        beta[tb * a.nR + k] = make_double2(s1 - (double)acc3[j][i], s1 + (double)acc2[j][i]);
      }
    }
  }
  if (KS) {
    // the split tiles: each wave's partial sums to LDS ([wave][value][lane], 16 KiB over the
    // tables and moments, which no wave reads any more), then added in wave order; KS = 1:
    // wave w finishes value w of the tile, KS = 2: wave w value pair (w & 1) of tile w >> 1
    constexpr int j = TW - 1;
    double2* sP = (double2*)lds_m2l;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double s1 = (double)acc1[j][i];
      sP[(w * 4 + i) * 64 + lane] = make_double2(s1 - (double)acc3[j][i], s1 + (double)acc2[j][i]);
    }
    __syncthreads();
    const int id = 4 * (TW - 1) + (KS == 1 ? 0 : (w >> 1));
    const int rb = id % a.nRB, cb = id / a.nRB;
    const int n = 16 * cb + col;
    if (id < ntile && ((tmask >> n) & 1)) {
      const int ix = px + 2 * (4 * X0 + (n & 3)), iy = py + 2 * (4 * NCB * Y0 + (n >> 2));
      const int64_t tb = ((int64_t)ix * N + iy) * N + iz;
#pragma unroll
      for (int q = 0; q < (KS == 1 ? 1 : 2); ++q) {
        const int i = KS == 1 ? w : 2 * (w & 1) + q;
        const int k = 16 * rb + Ty::row(krow, i);
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < (KS == 1 ? 4 : 2); ++u) {
          const int src = KS == 1 ? u : 2 * (w >> 1) + u;
          const double2 pv = sP[(src * 4 + i) * 64 + lane];
          v.x += pv.x, v.y += pv.y;
        }
        if (k < a.nR) beta[tb * a.nR + k] = v;
      }
    }
  }
}

template <typename T, int TW, int NCB>
static void (*pick_m2l(bool ex, int ks))(M2LArgs) {
  if (ks == 1) return k_m2l<T, TW, NCB, false, 1>;
  if (ks == 2) return k_m2l<T, TW, NCB, false, 2>;
  return ex ? k_m2l<T, TW, NCB, true, 0> : k_m2l<T, TW, NCB, false, 0>;
}

template <typename T, int NCB>
static hipError_t launch_t2(const M2LArgs& a0, int nrhs, hipStream_t s) {
  typedef typename M2LTypes<T>::T2 T2;
  M2LArgs a = a0;
  int total = 0;
  for (int i = 0; i < a.nlev; ++i) {
    M2LLevel& L = a.lev[i];
    L.tiles_x = ((L.n / 2) + 3) / 4;
    L.tiles_y = ((L.n / 2) + 4 * NCB - 1) / (4 * NCB);
    L.ntiles = L.n * 4 * L.tiles_x * L.tiles_y;
    a.tile_start[i] = total;
    total += (i == a.nlev - 1) ? 8 * ((L.ntiles + 7) / 8) : L.ntiles;
  }
  a.tile_start[a.nlev] = total;
  // stage the source moments in two phases when that lets two workgroups share a CU
  auto lds_of = [&](int kpb) {
    int rs = 4 * kpb;
    while (rs % 16 != 1) ++rs;
    return std::make_pair(((size_t)3 * a.P2 * a.P2 + 1) * sizeof(T2) + (size_t)16 * NCB * rs * sizeof(T2) +
                              4 * (size_t)a.nKB * sizeof(int) + (size_t)13 * (8 * NCB + 5) * 7, rs);
  };
  const int kpb1 = a.nKB, kpb2 = (a.nKB + 1) / 2;
  a.kph = (lds_of(kpb1).first > 80 * 1024 && lds_of(kpb2).first <= 80 * 1024) ? 2 : 1;
  a.kpb = a.kph == 1 ? kpb1 : kpb2;
  if (a.kph == 2 && a.nR % 2 == 0) {
    // blocks per phase rounded up so that each thread stages a run of 2, 4, 6 or 8 entries
    const int m = NCB == 1 ? 8 : 4, up = (a.kpb + m - 1) / m * m;
    if (NCB * up / 4 <= 8 && lds_of(up).first <= 80 * 1024) a.kpb = up;
  }
  const size_t lds = lds_of(a.kpb).first;
  a.nRsP = lds_of(a.kpb).second;
  const int ntile = a.nRB * NCB, TW = (ntile + 3) / 4, rem = ntile % 4;
  const bool ex = rem == 0;
  // one or two tiles left over: split along K over the waves (the partial sums need 16 KiB of LDS)
  const int ks = a.ksplit && (rem == 1 || rem == 2) && lds >= 16384 ? rem : 0;
  if (a.nsplit < 1) a.nsplit = 1;
  dim3 grid(total, nrhs, a.nsplit), block(256);
  void (*fn)(M2LArgs) = nullptr;
  switch (TW) {
    case 1: fn = pick_m2l<T, 1, NCB>(ex, ks); break;
    case 2: fn = pick_m2l<T, 2, NCB>(ex, ks); break;
    case 3: fn = pick_m2l<T, 3, NCB>(ex, ks); break;
    case 4: fn = pick_m2l<T, 4, NCB>(ex, ks); break;
    case 5: fn = pick_m2l<T, 5, NCB>(ex, ks); break;
    case 6: fn = pick_m2l<T, 6, NCB>(ex, ks); break;
    case 7: fn = pick_m2l<T, 7, NCB>(ex, ks); break;
    case 8: fn = pick_m2l<T, 8, NCB>(ex, ks); break;
    case 9: fn = pick_m2l<T, 9, NCB>(ex, ks); break;
    case 10: fn = pick_m2l<T, 10, NCB>(ex, ks); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, grid, block, lds, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(const M2LArgs& a, int nrhs, hipStream_t s) {
  typedef typename M2LTypes<T>::T2 T2;
  // 32 targets per workgroup when the widest level is wide enough and two
  // workgroups still fit in the LDS of a CU; 16 otherwise.
  const size_t lds2 = ((size_t)3 * a.P2 * a.P2 + 1) * sizeof(T2) + (size_t)32 * a.nRs * sizeof(T2);
  const int tw2 = (a.nRB * 2 + 3) / 4;
  const bool fit2 = lds2 <= 150 * 1024 && tw2 <= 10;
  if (a.ncb == 2 && fit2) return launch_t2<T, 2>(a, nrhs, s);
  if (a.ncb == 1) return launch_t2<T, 1>(a, nrhs, s);
  if (a.lev[a.nlev - 1].n >= 16 && lds2 <= 78 * 1024 && tw2 <= 10) return launch_t2<T, 2>(a, nrhs, s);
  return launch_t2<T, 1>(a, nrhs, s);
}

// ---------------------------------------------------------------------------
// Cross-layer M2L (Algorithm 2, components with target and source in different
// layers).  Moments and locals are used in the z-reduced form (k3 <= 1) so that
// only the z' derivative orders 0 and 1 of the kernel are needed; for those the
// source height enters through per-height complex images (Sec. 3.3).  The table
// of key (dx, dy, iz_t, iz_s) and order k3' holds
//   (-1)^{k3'} h^{k3'} h^{|g|} D^g [d^{k3'}_{z'} G / k3'!]
// in the frame (z, y, x) (entries with small z order), so that
//   b_k = sum_{k'} T^{(k3')}_{(k1+k1', k2+k2', k3)} a_{k'}
// with a the z-reduced scaled moments of the source box.  The target tile is
// a 4 x 4 NCB patch of boxes at one z index and one parity class; its list of
// (source group, dx, dy, iz_s, key) entries is built on the host from the
// acceptance test and is the same for every tile of the class.
// ---------------------------------------------------------------------------
template <typename T, int TW, int NCB>
__global__ __launch_bounds__(256) void k_m2l_cross(M2LCrossArgs a) {
  typedef M2LTypes<T> Ty;
  typedef typename Ty::T2 T2;
  typedef typename Ty::acc AC;
  constexpr int NT = 16 * NCB;
  extern __shared__ double lds_x[];
  const int P2 = a.P2;
  const int sub = 2 * P2 * P2;  // one k3' table: planes k3 = 0, 1
  T2* sG = (T2*)lds_x;          // [2 sub]
  T2* sA = sG + 2 * sub;        // [NT nRs]
  int* sCol = (int*)(sA + NT * a.nRs);

  int li = 0, tile = 0;
  const int widest = a.nlev - 1;
  if ((int)blockIdx.x < a.tile_start[widest]) {
    while ((int)blockIdx.x >= a.tile_start[li + 1]) ++li;
    tile = blockIdx.x - a.tile_start[li];
  } else {
    li = widest;
    const int b = blockIdx.x - a.tile_start[widest];
    const int nt = a.lev[li].ntiles;
    const int per = (nt + 7) / 8;
    tile = (b % 8) * per + b / 8;
    if (tile >= nt) return;
  }
  const M2LCrossLevel& L = a.lev[li];
  const int r = blockIdx.y, split = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  int t = tile;
  const int X0 = t % L.tiles_x;
  t /= L.tiles_x;
  const int Y0 = t % L.tiles_y;
  t /= L.tiles_y;
  const int px = t & 1, py = (t >> 1) & 1, iz = t >> 2;
  const int N = L.n;
  unsigned tmask = 0;
  for (int n = 0; n < NT; ++n) {
    const int ix = px + 2 * (4 * X0 + (n & 3)), iy = py + 2 * (4 * NCB * Y0 + (n >> 2));
    if (ix < N && iy < N) tmask |= 1u << n;
  }
  for (int e = tid; e < NT * a.nRs; e += 256) {
    sA[e].x = 0;
    sA[e].y = 0;
  }
  for (int e = tid; e < 2 * sub; e += 256) {
    sG[e].x = 0;
    sG[e].y = 0;
  }
  for (int e = tid; e < 4 * a.nKB; e += 256) {
    int v = 0;
    if (e < a.nR) {
      const int pk = a.rzmi[e];
      const int k1 = pk & 255, k2 = (pk >> 8) & 255, k3 = pk >> 16;
      v = (k3 * sub + (k1 + k2) * P2 + k1) | (1 << 24);
    }
    sCol[e] = v;
  }
  const int col = lane & 15, krow = lane >> 4;
  const int ntile = a.nRB * NCB;
  int rowo[TW], tcb[TW];
#pragma unroll
  for (int j = 0; j < TW; ++j) {
    const int id = w + 4 * j;
    const int rb = id % a.nRB, cb = id / a.nRB;
    const int k = 16 * rb + col;
    // rows past nR (and missing tiles) gather entry 0: finite, and dropped by the epilogue
    rowo[j] = 0, tcb[j] = cb;
    if (id < ntile && k < a.nR) {
      const int pk = a.rzmi[k];
      const int k1 = pk & 255, k2 = (pk >> 8) & 255, k3 = pk >> 16;
      rowo[j] = (k3 * P2 + k1 + k2) * P2 + k1;
    }
  }
  // B operand offset of each tile (column block tcb, target col); complex products by
  // three real products, as in k_m2l
  constexpr bool BT = TW <= 2;
  int boff[TW];
#pragma unroll
  for (int j = 0; j < TW; ++j) boff[j] = (16 * tcb[j] + col) * a.nRs;
  AC acc1[TW], acc2[TW], acc3[TW];
#pragma unroll
  for (int j = 0; j < TW; ++j) {
    acc1[j] = AC{0, 0, 0, 0};
    acc2[j] = AC{0, 0, 0, 0};
    acc3[j] = AC{0, 0, 0, 0};
  }
  // staging walk: element e = tid + 256 i of the NT x nR block is (n, kk), advanced by
  // 256 = q nR + rem per step
  const int n0 = tid / a.nR, kk0 = tid - n0 * a.nR;
  const int step_q = 256 / a.nR, step_r = 256 - step_q * a.nR;
  const int cls = 4 * iz + px + 2 * py;
  const int e0 = L.list_start[cls], e1 = L.list_start[cls + 1];
  for (int ei = e0 + split; ei < e1; ei += a.nsplit) {
    const CrossEntry ce = L.list[ei];
    unsigned smask = 0;
    for (int n = 0; n < NT; ++n) {
      const int ix = px + 2 * (4 * X0 + (n & 3)) + ce.dx, iy = py + 2 * (4 * NCB * Y0 + (n >> 2)) + ce.dy;
      if (((tmask >> n) & 1) && ix >= 0 && iy >= 0 && ix < N && iy < N) smask |= 1u << n;
    }
    if (!smask) continue;
    const double2* asrc = ce.src == 0 ? L.asrc[0] : ce.src == 1 ? L.asrc[1] : ce.src == 2 ? L.asrc[2] : L.asrc[3];
    const int64_t sst = ce.src == 0 ? L.src_stride[0]
                        : ce.src == 1 ? L.src_stride[1]
                        : ce.src == 2 ? L.src_stride[2]
                                      : L.src_stride[3];
    const double2* alpha = asrc + (int64_t)r * sst;
    __syncthreads();
    for (int kk3 = 0; kk3 < 2; ++kk3) {
      const T2* g = (const T2*)(sizeof(T) == 8 ? (const void*)L.T[kk3] : (const void*)L.T32[kk3]) +
                    (int64_t)ce.key * a.nG;
      for (int e = tid; e < a.nG; e += 256) {
        const int pos = a.gpadz[e];
        if (pos >= 0) sG[kk3 * sub + pos] = g[e];
      }
    }
    {
      int n = n0, kk = kk0;
      for (int e = tid; e < NT * a.nR; e += 256) {
        T2 v;
        v.x = 0;
        v.y = 0;
        if ((smask >> n) & 1) {
          const int ix = px + 2 * (4 * X0 + (n & 3)) + ce.dx, iy = py + 2 * (4 * NCB * Y0 + (n >> 2)) + ce.dy;
          const int64_t sb = ((int64_t)ix * N + iy) * N + ce.izs;
          v = Ty::cvt(alpha[sb * a.nR + kk]);
        }
        sA[n * a.nRs + kk] = v;
        n += step_q, kk += step_r;
        if (kk >= a.nR) kk -= a.nR, ++n;
      }
    }
    __syncthreads();
    // operands of block kb (column offset 0 past nR, where the staged moments are zero);
    // those of the next block are loaded while the MFMAs of this one run
    auto load = [&](int kb, T2 (&bb)[TW], T2 (&g)[TW]) {
      const int kp = 4 * kb + krow;
      const int co = sCol[kp] & 0xFFFFFF;
      if (BT) {
#pragma unroll
        for (int j = 0; j < TW; ++j) bb[j] = sA[boff[j] + kp];
      } else {
        bb[0] = sA[col * a.nRs + kp];
        if (NCB == 2) bb[1] = sA[(16 + col) * a.nRs + kp];
      }
#pragma unroll
      for (int j = 0; j < TW; ++j) g[j] = sG[rowo[j] + co];
    };
    auto mma = [&](const T2 (&bb)[TW], const T2 (&g)[TW]) {
      constexpr int NB = BT ? TW : NCB;
      auto bsel = [&](const T (&v)[NB], int j) { return BT ? v[j] : (NCB == 2 && tcb[j] ? v[NB - 1] : v[0]); };
      T bc[NB], dmc[NB], cpd[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) bc[u] = bb[u].x, dmc[u] = bb[u].y - bb[u].x, cpd[u] = bb[u].x + bb[u].y;
#pragma unroll
      for (int j = 0; j < TW; ++j)
        if (w + 4 * j < ntile) acc1[j] = Ty::mfma(g[j].x + g[j].y, bsel(bc, j), acc1[j]);
#pragma unroll
      for (int j = 0; j < TW; ++j)
        if (w + 4 * j < ntile) acc2[j] = Ty::mfma(g[j].x, bsel(dmc, j), acc2[j]);
#pragma unroll
      for (int j = 0; j < TW; ++j)
        if (w + 4 * j < ntile) acc3[j] = Ty::mfma(g[j].y, bsel(cpd, j), acc3[j]);
    };
    T2 b1[TW], g1[TW], b2[TW], g2[TW];
    load(0, b1, g1);
    for (int kb = 0; kb < a.nKB; kb += 2) {
      if (kb + 1 < a.nKB) load(kb + 1, b2, g2);
      mma(b1, g1);
      if (kb + 1 >= a.nKB) break;
      if (kb + 2 < a.nKB) load(kb + 2, b1, g1);
      mma(b2, g2);
    }
  }
  double2* beta = L.b + (int64_t)split * L.split_stride + (int64_t)r * L.rhs_stride;
#pragma unroll
  for (int j = 0; j < TW; ++j) {
    const int id = w + 4 * j;
    if (id >= ntile) continue;
    const int rb = id % a.nRB, cb = id / a.nRB;
    const int n = 16 * cb + col;
    if (!((tmask >> n) & 1)) continue;
    const int ix = px + 2 * (4 * X0 + (n & 3)), iy = py + 2 * (4 * NCB * Y0 + (n >> 2));
    const int64_t tb = ((int64_t)ix * N + iy) * N + iz;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 16 * rb + Ty::row(krow, i);
      if (k < a.nR) {
        const double s1 = (double)acc1[j][i];
        beta[tb * a.nR + k] = make_double2(s1 - (double)acc3[j][i], s1 + (double)acc2[j][i]);
      }
    }
  }
}

template <typename T, int NCB>
static hipError_t launch_cross_t2(const M2LCrossArgs& a0, int nrhs, hipStream_t s) {
  typedef typename M2LTypes<T>::T2 T2;
  M2LCrossArgs a = a0;
  int total = 0;
  for (int i = 0; i < a.nlev; ++i) {
    M2LCrossLevel& L = a.lev[i];
    L.tiles_x = ((L.n / 2) + 3) / 4;
    L.tiles_y = ((L.n / 2) + 4 * NCB - 1) / (4 * NCB);
    L.ntiles = L.n * 4 * L.tiles_x * L.tiles_y;
    a.tile_start[i] = total;
    total += (i == a.nlev - 1) ? 8 * ((L.ntiles + 7) / 8) : L.ntiles;
  }
  a.tile_start[a.nlev] = total;
  const size_t lds = (size_t)4 * a.P2 * a.P2 * sizeof(T2) + (size_t)16 * NCB * a.nRs * sizeof(T2) +
                     4 * (size_t)a.nKB * sizeof(int);
  const int TW = (a.nRB * NCB + 3) / 4;
  if (a.nsplit < 1) a.nsplit = 1;
  dim3 grid(total, nrhs, a.nsplit), block(256);
  void (*fn)(M2LCrossArgs) = nullptr;
  switch (TW) {
    case 1: fn = k_m2l_cross<T, 1, NCB>; break;
    case 2: fn = k_m2l_cross<T, 2, NCB>; break;
    case 3: fn = k_m2l_cross<T, 3, NCB>; break;
    case 4: fn = k_m2l_cross<T, 4, NCB>; break;
    case 5: fn = k_m2l_cross<T, 5, NCB>; break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, grid, block, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_m2l_cross(const M2LCrossArgs& a, int nrhs, bool fp32, hipStream_t s) {
  if (a.nlev < 1 || a.nlev > M2L_MAX_LEVELS) return hipErrorInvalidValue;
  return fp32 ? launch_cross_t2<float, 1>(a, nrhs, s) : launch_cross_t2<double, 1>(a, nrhs, s);
}

hipError_t launch_m2l(const M2LArgs& a, int nrhs, bool fp32, hipStream_t s) {
  if (a.nlev < 1 || a.nlev > M2L_MAX_LEVELS) return hipErrorInvalidValue;
  return fp32 ? launch_t<float>(a, nrhs, s) : launch_t<double>(a, nrhs, s);
}

}  // namespace tefmm
