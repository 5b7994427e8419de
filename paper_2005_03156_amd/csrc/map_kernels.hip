// Point -> block mapping kernels for gfx950 (wave64).
//
// One kernel does the whole path for a tile of 64 points per wavefront:
//   1. hierarchical box filter (paper Sec. III): every point is tested
//      against the level-0 boxes (staged in LDS, same box for all lanes),
//      then against the children of each surviving group, level by level.
//      Survivors of each level are compacted into a per-wave LDS list of
//      (node, point) items with a wavefront ballot + mbcnt prefix count.
//   2. crossing-number test (paper Sec. III-A) on every surviving
//      (block, point) pair, edge-parallel: each pair's ring is cut into
//      chunks of a few edges, the chunks of all pairs of the tile are dealt
//      across the 64 lanes, and each chunk's crossing parity is folded into
//      its pair with an LDS xor.
//   3. result: for every pair with odd parity, atomic min of the block index
//      into the point's LDS slot; one coalesced store per tile.
// A point whose candidates would overflow a per-wave list (only for heavily
// overlapping input) is finished by a per-lane depth-first walk instead,
// which gives the same exact answer.
#include <hip/hip_runtime.h>

#include "common.h"

namespace bm {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kCap = 256;       // (node, point) items per list per wave
constexpr int kCapChunk = 512;  // crossing-test chunks per window per wave
constexpr int kL0Lds = 512;     // level-0 boxes staged in LDS when g0 fits

struct WaveLds {
  int2 pts[kWave];
  unsigned best[kWave];
  unsigned char ovf[kWave];
  unsigned node[2][kCap];
  unsigned char lane[2][kCap];
  unsigned parity[kCap];
  unsigned long long chunk0[kCap];
  unsigned short ch_pair[kCapChunk];
  unsigned ch_k[kCapChunk];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned long long t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ bool in_box(const int4& b, int2 p) {
  return b.x <= p.x && p.x < b.y && b.z <= p.y && p.y < b.w;
}

// Crossing of the ray from p towards +x with the edge a -> b.
// Takes part when exactly one end is strictly above p; counts when the edge
// meets the line y = p.y strictly right of p. With the x-range known:
// p.x < min(a.x, b.x) always crosses, p.x >= max(a.x, b.x) never does, and
// in between the sign of the 64-bit cross product
//   c = (a.x - p.x)(b.y - p.y) - (b.x - p.x)(a.y - p.y)
// decides (c > 0 for an upward edge, c < 0 for a downward one). There p lies
// inside the edge's box, so every factor is below 2^31 in magnitude and c
// fits in int64.
__device__ __forceinline__ unsigned crosses(int2 a, int2 b, int2 p) {
  const bool a_up = a.y > p.y, b_up = b.y > p.y;
  const int xlo = min(a.x, b.x), xhi = max(a.x, b.x);
  unsigned r = (a_up != b_up) & (p.x < xlo);
  const bool amb = (a_up != b_up) & (p.x >= xlo) & (p.x < xhi);
  if (amb) {
    const long long c = (long long)(a.x - p.x) * (long long)(b.y - p.y) -
                        (long long)(b.x - p.x) * (long long)(a.y - p.y);
    r = b_up ? (c > 0) : (c < 0);
  }
  return r;
}

// Full crossing-number test of one ring (stored closed).
__device__ unsigned ring_parity(const KIndex& ix, int leaf, int2 p) {
  const long long v0 = ix.vert_off[leaf], v1 = ix.vert_off[leaf + 1] - 1;
  unsigned acc = 0;
  int2 a = ix.verts[v0];
  for (long long j = v0; j < v1; ++j) {
    const int2 b = ix.verts[j + 1];
    acc ^= crosses(a, b, p);
    a = b;
  }
  return acc;
}

// Depth-first walk of the whole hierarchy for one point: used only for points
// whose candidate lists overflowed. Stackless: a node's parent link gives the
// way back up.
__device__ unsigned walk_point(const KIndex& ix, int2 p) {
  unsigned best = 0xFFFFFFFFu;
  int e = 0, end = ix.g0, par = -1;
  for (;;) {
    if (e >= end) {
      if (par < 0) break;
      e = par + 1;
      par = ix.parent[par];
      end = par < 0 ? ix.g0 : ix.child[par].y;
      continue;
    }
    if (in_box(ix.box[e], p)) {
      if (e >= ix.leaf_base) {
        const int leaf = e - ix.leaf_base;
        if (ring_parity(ix, leaf, p)) best = min(best, (unsigned)ix.leaf_id[leaf]);
        ++e;
      } else {
        const int2 c = ix.child[e];
        par = e;
        e = c.x;
        end = c.y;
      }
    } else {
      ++e;
    }
  }
  return best;
}

// Append (node, point lane) to list `dst` (wave-uniform count `cnt`) for
// every lane where `pred` holds; all 64 lanes must be active. Items that do
// not fit mark their point for the depth-first fallback.
__device__ __forceinline__ void emit(WaveLds& S, int dst, bool pred, unsigned node, int plane,
                                     unsigned& cnt) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const unsigned slot = cnt + lanes_below(m);
  if (pred) {
    if (slot < (unsigned)kCap) {
      S.node[dst][slot] = node;
      S.lane[dst][slot] = (unsigned char)plane;
    } else {
      S.ovf[plane] = 1;
    }
  }
  cnt += (unsigned)__popcll(m);
}

template <int kChunkShift>
__global__ __launch_bounds__(kBlock) void map_kernel(const KIndex ix, const int2* __restrict__ xy,
                                                     const long long n, int* __restrict__ out) {
  constexpr unsigned kChunk = 1u << kChunkShift;
  __shared__ int4 l0box[kL0Lds];
  __shared__ WaveLds wl[kWavesPerBlock];

  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  WaveLds& S = wl[w];
  const bool l0_lds = ix.g0 <= kL0Lds;
  if (l0_lds)
    for (int i = threadIdx.x; i < ix.g0; i += kBlock) l0box[i] = ix.box[i];
  __syncthreads();

  const long long ntiles = (n + kWave - 1) / kWave;
  const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
  for (long long t = (long long)blockIdx.x * kWavesPerBlock + w; t < ntiles; t += nwaves) {
    const long long i = t * kWave + lane;
    const bool valid = i < n;
    const int2 p = valid ? xy[i] : make_int2(0, 0);
    S.pts[lane] = p;
    S.best[lane] = 0xFFFFFFFFu;
    S.ovf[lane] = 0;
    wave_sync();

    // ---- level 0: every point against every level-0 box (uniform loop)
    int cur = 0;
    unsigned cnt = 0;
    for (int j = 0; j < ix.g0; ++j) {
      const int4 b = l0_lds ? l0box[j] : ix.box[j];
      emit(S, cur, valid && in_box(b, p), (unsigned)j, lane, cnt);
    }
    cnt = min(cnt, (unsigned)kCap);
    wave_sync();

    // ---- lower levels: children of the surviving groups
    for (int l = 0; l < ix.n_levels; ++l) {
      const int nxt = cur ^ 1;
      unsigned ncnt = 0;
      for (unsigned r = 0; r < cnt; r += kWave) {
        const unsigned q = r + lane;
        const bool has = q < cnt;
        const unsigned node = has ? S.node[cur][q] : 0u;
        const int pl = has ? S.lane[cur][q] : 0;
        const int2 cr = has ? ix.child[node] : make_int2(0, 0);
        const int2 pp = S.pts[pl];
        const int len = cr.y - cr.x;
        const int maxlen = wave_max(len);
        for (int k = 0; k < maxlen; ++k) {
          const bool act = k < len;
          const int c = cr.x + (act ? k : 0);
          const bool in = act && in_box(ix.box[act ? c : 0], pp);
          emit(S, nxt, in, (unsigned)c, pl, ncnt);
        }
      }
      cnt = min(ncnt, (unsigned)kCap);
      cur = nxt;
      wave_sync();
    }

    // ---- crossing-number test on the (leaf, point) pairs in list `cur`
    unsigned long long total = 0;
    for (unsigned r = 0; r < cnt; r += kWave) {
      const unsigned q = r + lane;
      const bool has = q < cnt;
      unsigned long long nch = 0;
      if (has) {
        const int leaf = (int)S.node[cur][q] - ix.leaf_base;
        const long long edges = ix.vert_off[leaf + 1] - ix.vert_off[leaf] - 1;
        nch = (unsigned long long)((edges + kChunk - 1) >> kChunkShift);
      }
      const unsigned long long incl = wave_incl_scan(nch, lane);
      if (has) {
        S.chunk0[q] = total + incl - nch;
        S.parity[q] = 0;
      }
      total += __shfl(incl, kWave - 1);
    }
    wave_sync();

    for (unsigned long long wlo = 0; wlo < total; wlo += kCapChunk) {
      const unsigned long long whi = min(wlo + (unsigned long long)kCapChunk, total);
      // deal this window's chunks: pair q owns chunk ids [chunk0[q], chunk0[q+1])
      for (unsigned r = 0; r < cnt; r += kWave) {
        const unsigned q = r + lane;
        if (q < cnt) {
          const unsigned long long c0 = S.chunk0[q];
          const unsigned long long c1 = (q + 1 < cnt) ? S.chunk0[q + 1] : total;
          const unsigned long long a = max(c0, wlo), b = min(c1, whi);
          for (unsigned long long c = a; c < b; ++c) {
            S.ch_pair[c - wlo] = (unsigned short)q;
            S.ch_k[c - wlo] = (unsigned)(c - c0);
          }
        }
      }
      wave_sync();
      const unsigned nwin = (unsigned)(whi - wlo);
      for (unsigned c = lane; c < nwin; c += kWave) {
        const unsigned q = S.ch_pair[c];
        const unsigned k = S.ch_k[c];
        const int leaf = (int)S.node[cur][q] - ix.leaf_base;
        const int2 pp = S.pts[S.lane[cur][q]];
        const long long v0 = ix.vert_off[leaf];
        const long long vlast = ix.vert_off[leaf + 1] - 1;  // index of the closing copy
        const long long j0 = v0 + ((long long)k << kChunkShift);
        const long long j1 = min(j0 + (long long)kChunk, vlast);
        int2 a = ix.verts[j0];
        unsigned acc = 0;
        for (long long j = j0; j < j1; ++j) {
          const int2 b = ix.verts[j + 1];
          acc ^= crosses(a, b, pp);
          a = b;
        }
        if (acc) atomicXor(&S.parity[q], 1u);
      }
      wave_sync();
    }

    for (unsigned r = 0; r < cnt; r += kWave) {
      const unsigned q = r + lane;
      if (q < cnt && (S.parity[q] & 1u)) {
        const int leaf = (int)S.node[cur][q] - ix.leaf_base;
        atomicMin(&S.best[S.lane[cur][q]], (unsigned)ix.leaf_id[leaf]);
      }
    }
    wave_sync();

    unsigned best = S.best[lane];
    if (valid && S.ovf[lane]) best = min(best, walk_point(ix, p));
    if (valid) out[i] = (int)best;
    wave_sync();
  }
}

// Quantiser: q = rint(v * 2^22) + 2^30 per axis; invalid input -> (-1, -1).
// The product by a power of two is exact, so rint is the only rounding.
__global__ __launch_bounds__(256) void quantize_kernel(const double2* __restrict__ ll,
                                                       const long long n, int2* __restrict__ xy) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double2 v = ll[i];
    const bool ok = (fabs(v.x) <= 180.0) && (fabs(v.y) <= 90.0);  // false for NaN
    const long long qx = (long long)rint(v.x * 4194304.0) + 1073741824ll;
    const long long qy = (long long)rint(v.y * 4194304.0) + 1073741824ll;
    xy[i] = ok ? make_int2((int)qx, (int)qy) : make_int2(-1, -1);
  }
}

}  // namespace

hipError_t launch_map(const KIndex& ix, const int32_t* xy, int64_t n, int32_t* out,
                      const Tuning& t, int num_cu, hipStream_t stream) {
  const long long tiles = (n + kWave - 1) / kWave;
  long long blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  const long long cap = (long long)num_cu * t.blocks_per_cu;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(kBlock);
  const int2* p = reinterpret_cast<const int2*>(xy);
  switch (t.edge_chunk) {
    case 4:
      hipLaunchKernelGGL(map_kernel<2>, grid, block, 0, stream, ix, p, (long long)n, out);
      break;
    case 16:
      hipLaunchKernelGGL(map_kernel<4>, grid, block, 0, stream, ix, p, (long long)n, out);
      break;
    default:
      hipLaunchKernelGGL(map_kernel<3>, grid, block, 0, stream, ix, p, (long long)n, out);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_quantize(const double* lonlat, int64_t n, int32_t* xy, int num_cu,
                           hipStream_t stream) {
  long long blocks = (n + 255) / 256;
  const long long cap = (long long)num_cu * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                     reinterpret_cast<const double2*>(lonlat), (long long)n,
                     reinterpret_cast<int2*>(xy));
  return hipGetLastError();
}

}  // namespace bm
