// Index construction: validation, node ordering, half-open boxes, upload.
//
// The hierarchy of the paper (Sec. III-B: states holding counties holding
// blocks, each with a bounding box and, for blocks, a polygon) becomes one
// node array on the device. Nodes are renumbered level by level so that the
// children of every group are contiguous (a stable counting sort on the
// parent's new position); leaves keep their caller-given block index in
// leaf_id. Leaf boxes are the half-open extent of their ring; a group's box is
// the smallest box holding its children's boxes, so the filter never loses a
// containing block whatever the grouping.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace bm {
namespace {

constexpr int kTableMinChildren = 6;  // below this a group's children are simply all tested

struct HostIndex {
  int32_t n_levels = 0, g0 = 0, leaf_base = 0, n_leaves = 0;
  int4 root_child = {0, 0, -1, 0};
  int4 root_box = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
  std::vector<int4> box;
  std::vector<int4> child;
  std::vector<uint64_t> slot_mask;
  std::vector<int32_t> parent;
  std::vector<int64_t> vert_off;
  std::vector<int32_t> leaf_id;
  std::vector<int2> verts;
};

// Slot table of a group with 6..64 children: the group box is cut into S
// equal power-of-two slots per axis (S = 8 up to 16 children, else 16), and
// slot s of an axis holds a bit for every child whose box overlaps it on that
// axis. For a point in the group box, (x-slot mask & y-slot mask) is a superset
// of the children whose boxes contain it; the exact half-open box test is then
// run on those children only, so the filter's result is unchanged.
int4 make_table(const std::vector<int4>& box, int c0, int c1, const int4& g,
                std::vector<uint64_t>& masks) {
  int4 r = make_int4(c0, c1, -1, 0);
  const int m = c1 - c0;
  if (m < kTableMinChildren || m > 64 || g.x >= g.y || g.z >= g.w) return r;
  const int logS = m <= 16 ? 3 : 4, S = 1 << logS;
  const int64_t wx = (int64_t)g.y - g.x, wy = (int64_t)g.w - g.z;
  int shx = 0, shy = 0;
  while (((int64_t)S << shx) < wx) ++shx;
  while (((int64_t)S << shy) < wy) ++shy;
  const size_t off = masks.size();
  if (off + 2 * S > (size_t)INT32_MAX) return r;
  masks.resize(off + 2 * S, 0);
  for (int c = c0; c < c1; ++c) {
    const int4 b = box[c];
    if (b.x >= b.y || b.z >= b.w) continue;  // an empty box holds no point
    const uint64_t bit = 1ull << (c - c0);
    const int64_t sx0 = ((int64_t)b.x - g.x) >> shx, sx1 = ((int64_t)b.y - 1 - g.x) >> shx;
    const int64_t sy0 = ((int64_t)b.z - g.z) >> shy, sy1 = ((int64_t)b.w - 1 - g.z) >> shy;
    for (int64_t t = sx0; t <= sx1; ++t) masks[off + t] |= bit;
    for (int64_t t = sy0; t <= sy1; ++t) masks[off + S + t] |= bit;
  }
  r.z = (int)off;
  r.w = logS | (shx << 8) | (shy << 16);
  return r;
}

int build_host(const bm_index_desc* d, HostIndex& h) {
  if (!d) return fail(BM_EINVAL, "bm_index_create: null descriptor");
  const int64_t B = d->n_blocks;
  if (B < 0 || B > INT32_MAX) return fail(BM_EINVAL, "bm_index_create: n_blocks out of range");
  if (d->n_levels < 0 || d->n_levels > 64) return fail(BM_EINVAL, "bm_index_create: n_levels out of range");
  if (B > 0 && (!d->vert_off || !d->verts_xy)) return fail(BM_EINVAL, "bm_index_create: null ring arrays");
  const int L = d->n_levels;
  if (L > 0 && (!d->n_groups || !d->parent)) return fail(BM_EINVAL, "bm_index_create: null hierarchy arrays");

  // level sizes, coarse to fine; the last level is the blocks
  std::vector<int64_t> size(L + 1);
  int64_t total_nodes = 0;
  for (int l = 0; l < L; ++l) {
    if (d->n_groups[l] < 1 || d->n_groups[l] > INT32_MAX)
      return fail(BM_EINVAL, "bm_index_create: n_groups[" + std::to_string(l) + "] out of range");
    if (!d->parent[l]) return fail(BM_EINVAL, "bm_index_create: null parent[" + std::to_string(l) + "]");
    size[l] = d->n_groups[l];
    total_nodes += size[l];
  }
  size[L] = B;
  total_nodes += B;
  if (total_nodes > INT32_MAX) return fail(BM_ERANGE, "bm_index_create: too many nodes");

  // rings
  if (B > 0) {
    if (d->vert_off[0] != 0) return fail(BM_EINVAL, "bm_index_create: vert_off[0] must be 0");
    for (int64_t b = 0; b < B; ++b) {
      const int64_t m = d->vert_off[b + 1] - d->vert_off[b];
      if (m < 3)
        return fail(BM_EINVAL, "bm_index_create: ring " + std::to_string(b) + " has fewer than 3 vertices");
    }
    const int64_t V = d->vert_off[B];
    for (int64_t k = 0; k < 2 * V; ++k)
      if (d->verts_xy[k] < 0)
        return fail(BM_ERANGE, "bm_index_create: vertex coordinate outside [0, 2^31-1] at vertex " +
                                   std::to_string(k / 2));
  }
  // parents
  for (int l = 0; l < L; ++l) {
    const int32_t* par = d->parent[l];
    for (int64_t e = 0; e < size[l + 1]; ++e)
      if (par[e] < 0 || par[e] >= size[l])
        return fail(BM_EINVAL, "bm_index_create: parent[" + std::to_string(l) + "][" + std::to_string(e) +
                                   "] out of range");
  }

  // new positions: level 0 keeps its order; a finer level is sorted stably by
  // the new position of its parent
  std::vector<int64_t> base(L + 2, 0);
  for (int l = 0; l <= L; ++l) base[l + 1] = base[l] + size[l];
  std::vector<std::vector<int32_t>> pos(L + 1);   // pos[l][e] = new position within level
  std::vector<std::vector<int32_t>> order(L + 1); // order[l][new] = e
  pos[0].resize(size[0]);
  order[0].resize(size[0]);
  for (int64_t e = 0; e < size[0]; ++e) pos[0][e] = order[0][e] = (int32_t)e;
  h.child.assign(base[L], make_int4(0, 0, -1, 0));
  h.parent.assign(total_nodes, -1);
  for (int l = 0; l < L; ++l) {
    const int32_t* par = d->parent[l];
    const int64_t G = size[l], E = size[l + 1];
    std::vector<int64_t> cnt(G + 1, 0);
    for (int64_t e = 0; e < E; ++e) cnt[pos[l][par[e]] + 1]++;
    for (int64_t g = 0; g < G; ++g) cnt[g + 1] += cnt[g];
    for (int64_t g = 0; g < G; ++g)  // children of the group at new position g
      h.child[base[l] + g] = make_int4((int)(base[l + 1] + cnt[g]), (int)(base[l + 1] + cnt[g + 1]), -1, 0);
    pos[l + 1].resize(E);
    order[l + 1].resize(E);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
      const int64_t np = fill[pos[l][par[e]]]++;
      pos[l + 1][e] = (int32_t)np;
      order[l + 1][np] = (int32_t)e;
      h.parent[base[l + 1] + np] = (int32_t)(base[l] + pos[l][par[e]]);
    }
  }

  // leaves: rings in new order, each closed by a copy of its first vertex
  h.box.assign(total_nodes, make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN));
  h.vert_off.assign(B + 1, 0);
  h.leaf_id.assign(B, 0);
  for (int64_t nb = 0; nb < B; ++nb) {
    const int32_t b = order[L][nb];
    h.vert_off[nb + 1] = h.vert_off[nb] + (d->vert_off[b + 1] - d->vert_off[b]) + 1;
    h.leaf_id[nb] = b;
  }
  h.verts.resize(h.vert_off[B]);
  for (int64_t nb = 0; nb < B; ++nb) {
    const int32_t b = order[L][nb];
    const int32_t* src = d->verts_xy + 2 * d->vert_off[b];
    const int64_t m = d->vert_off[b + 1] - d->vert_off[b];
    int2* dst = h.verts.data() + h.vert_off[nb];
    int4 bx = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
    for (int64_t k = 0; k < m; ++k) {
      const int x = src[2 * k], y = src[2 * k + 1];
      dst[k] = make_int2(x, y);
      bx.x = std::min(bx.x, x);
      bx.y = std::max(bx.y, x);
      bx.z = std::min(bx.z, y);
      bx.w = std::max(bx.w, y);
    }
    dst[m] = dst[0];
    h.box[base[L] + nb] = bx;
  }
  // group boxes, finest group level first
  for (int l = L - 1; l >= 0; --l)
    for (int64_t g = 0; g < size[l]; ++g) {
      const int4 cr = h.child[base[l] + g];
      int4 bx = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
      for (int c = cr.x; c < cr.y; ++c) {
        const int4 s = h.box[c];
        bx.x = std::min(bx.x, s.x);
        bx.y = std::max(bx.y, s.y);
        bx.z = std::min(bx.z, s.z);
        bx.w = std::max(bx.w, s.w);
      }
      h.box[base[l] + g] = bx;
    }
  // slot tables: every group, then the virtual root over level 0
  for (int64_t g = 0; g < base[L]; ++g)
    h.child[g] = make_table(h.box, h.child[g].x, h.child[g].y, h.box[g], h.slot_mask);
  int4 rb = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
  for (int64_t e = 0; e < size[0]; ++e) {
    const int4 s = h.box[e];
    rb.x = std::min(rb.x, s.x);
    rb.y = std::max(rb.y, s.y);
    rb.z = std::min(rb.z, s.z);
    rb.w = std::max(rb.w, s.w);
  }
  h.root_box = rb;
  h.root_child = make_table(h.box, 0, (int)size[0], rb, h.slot_mask);
  h.n_levels = L;
  h.g0 = (int32_t)size[0];
  h.leaf_base = (int32_t)base[L];
  h.n_leaves = (int32_t)B;
  return BM_OK;
}

template <class T>
int upload(bm_index* ix, const std::vector<T>& v, const T** dst) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(v.size() * sizeof(T), sizeof(T));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    return fail(e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EHIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  ix->allocs[ix->n_allocs++] = p;
  ix->bytes += (int64_t)bytes;
  if (!v.empty()) {
    e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  *dst = static_cast<const T*>(p);
  return BM_OK;
}

void free_index(bm_index* ix) {
  if (!ix) return;
  for (int i = 0; i < ix->n_allocs; ++i) (void)hipFree(ix->allocs[i]);
  delete ix;
}

int make_device(HostIndex& h, bm_index** out) {
  bm_index* ix = new (std::nothrow) bm_index();
  if (!ix) return fail(BM_ENOMEM, "bm_index_create: host allocation failed");
  hipError_t e = hipGetDevice(&ix->device);
  if (e != hipSuccess) {
    delete ix;
    return fail(BM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  e = hipDeviceGetAttribute(&ix->num_cu, hipDeviceAttributeMultiprocessorCount, ix->device);
  if (e != hipSuccess || ix->num_cu < 1) ix->num_cu = 256;
  KIndex& k = ix->k;
  int rc = BM_OK;
  if (rc == BM_OK) rc = upload(ix, h.box, &k.box);
  if (rc == BM_OK) rc = upload(ix, h.child, &k.child);
  if (rc == BM_OK) rc = upload(ix, h.slot_mask, reinterpret_cast<const uint64_t**>(&k.slot_mask));
  if (rc == BM_OK) rc = upload(ix, h.parent, &k.parent);
  if (rc == BM_OK) rc = upload(ix, h.vert_off, &k.vert_off);
  if (rc == BM_OK) rc = upload(ix, h.leaf_id, &k.leaf_id);
  if (rc == BM_OK) rc = upload(ix, h.verts, &k.verts);
  if (rc != BM_OK) {
    free_index(ix);
    return rc;
  }
  k.n_levels = h.n_levels;
  k.root_child = h.root_child;
  k.root_box = h.root_box;
  k.g0 = h.g0;
  k.leaf_base = h.leaf_base;
  k.n_leaves = h.n_leaves;
  ix->n_blocks = h.n_leaves;
  ix->n_nodes = (int64_t)h.box.size();
  ix->n_verts_stored = (int64_t)h.verts.size();
  ix->n_masks = (int64_t)h.slot_mask.size();
  *out = ix;
  return BM_OK;
}

// ---- flat file: magic, version, scalars, then the six arrays
constexpr char kMagic[8] = {'B', 'M', 'I', 'D', 'X', '0', '0', '1'};

template <class T>
bool write_vec(FILE* f, const std::vector<T>& v) {
  const int64_t n = (int64_t)v.size();
  return fwrite(&n, sizeof n, 1, f) == 1 && (n == 0 || fwrite(v.data(), sizeof(T), n, f) == (size_t)n);
}

template <class T>
bool read_vec(FILE* f, std::vector<T>& v, int64_t max_n) {
  int64_t n = 0;
  if (fread(&n, sizeof n, 1, f) != 1 || n < 0 || n > max_n) return false;
  v.resize(n);
  return n == 0 || fread(v.data(), sizeof(T), n, f) == (size_t)n;
}

template <class T>
int download(const T* src, int64_t n, std::vector<T>& v) {
  v.resize(n);
  if (n == 0) return BM_OK;
  hipError_t e = hipMemcpy(v.data(), src, n * sizeof(T), hipMemcpyDeviceToHost);
  return e == hipSuccess ? BM_OK : fail(BM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
}

}  // namespace

int index_create(const bm_index_desc* d, bm_index** out) {
  if (!out) return fail(BM_EINVAL, "bm_index_create: null output pointer");
  *out = nullptr;
  HostIndex h;
  int rc = build_host(d, h);
  if (rc != BM_OK) return rc;
  return make_device(h, out);
}

void index_destroy(bm_index* ix) { free_index(ix); }

int index_save(const bm_index* ix, const char* path) {
  if (!ix || !path) return fail(BM_EINVAL, "bm_index_save: null argument");
  HostIndex h;
  const KIndex& k = ix->k;
  int rc = BM_OK;
  if (rc == BM_OK) rc = download(k.box, ix->n_nodes, h.box);
  if (rc == BM_OK) rc = download(k.child, (int64_t)k.leaf_base, h.child);
  if (rc == BM_OK) rc = download(reinterpret_cast<const uint64_t*>(k.slot_mask), ix->n_masks, h.slot_mask);
  if (rc == BM_OK) rc = download(k.parent, ix->n_nodes, h.parent);
  if (rc == BM_OK) rc = download(k.vert_off, (int64_t)k.n_leaves + 1, h.vert_off);
  if (rc == BM_OK) rc = download(k.leaf_id, (int64_t)k.n_leaves, h.leaf_id);
  if (rc == BM_OK) rc = download(k.verts, ix->n_verts_stored, h.verts);
  if (rc != BM_OK) return rc;
  FILE* f = fopen(path, "wb");
  if (!f) return fail(BM_EIO, std::string("bm_index_save: cannot open ") + path);
  const int32_t sc[12] = {k.n_levels, k.g0, k.leaf_base, k.n_leaves,
                          k.root_child.x, k.root_child.y, k.root_child.z, k.root_child.w,
                          k.root_box.x, k.root_box.y, k.root_box.z, k.root_box.w};
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(sc, sizeof sc, 1, f) == 1 && write_vec(f, h.box) &&
            write_vec(f, h.child) && write_vec(f, h.slot_mask) && write_vec(f, h.parent) &&
            write_vec(f, h.vert_off) &&
            write_vec(f, h.leaf_id) && write_vec(f, h.verts);
  ok = (fclose(f) == 0) && ok;
  return ok ? BM_OK : fail(BM_EIO, std::string("bm_index_save: write failed on ") + path);
}

int index_load(const char* path, bm_index** out) {
  if (!path || !out) return fail(BM_EINVAL, "bm_index_load: null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(BM_EIO, std::string("bm_index_load: cannot open ") + path);
  HostIndex h;
  char magic[8];
  int32_t sc[12];
  const int64_t lim = (int64_t)1 << 40;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(sc, sizeof sc, 1, f) == 1 &&
            read_vec(f, h.box, INT32_MAX) && read_vec(f, h.child, INT32_MAX) &&
            read_vec(f, h.slot_mask, INT32_MAX) && read_vec(f, h.parent, INT32_MAX) &&
            read_vec(f, h.vert_off, INT32_MAX) && read_vec(f, h.leaf_id, INT32_MAX) && read_vec(f, h.verts, lim);
  fclose(f);
  if (!ok) return fail(BM_EIO, std::string("bm_index_load: malformed file ") + path);
  h.n_levels = sc[0];
  h.g0 = sc[1];
  h.leaf_base = sc[2];
  h.n_leaves = sc[3];
  h.root_child = make_int4(sc[4], sc[5], sc[6], sc[7]);
  h.root_box = make_int4(sc[8], sc[9], sc[10], sc[11]);
  // structural checks so that a damaged file cannot send the kernels out of bounds
  const int64_t N = (int64_t)h.box.size();
  bool good = h.n_levels >= 0 && h.g0 >= 0 && h.leaf_base >= 0 && h.n_leaves >= 0 &&
              (int64_t)h.leaf_base + h.n_leaves == N && (int64_t)h.child.size() == h.leaf_base &&
              (int64_t)h.parent.size() == N && (int64_t)h.vert_off.size() == (int64_t)h.n_leaves + 1 &&
              (int64_t)h.leaf_id.size() == h.n_leaves && h.g0 <= N && (h.n_levels > 0 || h.g0 == h.n_leaves) &&
              (h.n_levels == 0 || h.g0 <= h.leaf_base);
  if (good && !h.vert_off.empty()) {
    good = h.vert_off[0] == 0 && h.vert_off.back() == (int64_t)h.verts.size();
    for (int64_t b = 0; good && b < h.n_leaves; ++b) good = h.vert_off[b + 1] - h.vert_off[b] >= 2;
  }
  auto table_ok = [&](const int4& c) {
    if (c.z < 0) return true;
    const int logS = c.w & 0xff, shx = (c.w >> 8) & 0xff, shy = (c.w >> 16) & 0xff, m = c.y - c.x;
    if ((logS != 3 && logS != 4) || shx > 31 || shy > 31 || m < 1 || m > 64) return false;
    const int64_t S = 1 << logS;
    if ((int64_t)c.z + 2 * S > (int64_t)h.slot_mask.size()) return false;
    const uint64_t keep = m == 64 ? ~0ull : ((1ull << m) - 1);
    for (int64_t t = 0; t < 2 * S; ++t)
      if (h.slot_mask[c.z + t] & ~keep) return false;
    return true;
  };
  for (int64_t g = 0; good && g < h.leaf_base; ++g)
    good = h.child[g].x >= 0 && h.child[g].x <= h.child[g].y && h.child[g].y <= N && h.child[g].x > g &&
           table_ok(h.child[g]);
  good = good && h.root_child.x == 0 && h.root_child.y == h.g0 && table_ok(h.root_child);
  for (int64_t e = 0; good && e < N; ++e) good = h.parent[e] >= -1 && h.parent[e] < N && h.parent[e] < e;
  if (!good) return fail(BM_EIO, std::string("bm_index_load: inconsistent index in ") + path);
  return make_device(h, out);
}

}  // namespace bm
