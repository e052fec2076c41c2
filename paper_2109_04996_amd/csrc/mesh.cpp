// Mesh ingestion: validation, element coloring and ordering, ownership masks.
//
// libCEED section (operator decomposition): the element restriction G maps the
// L-vector to per-element values through an index array; its transpose G^T
// sums element contributions back into the L-vector. The fused apply does
// G^T without atomics: elements are split into colors so that no two
// elements of one color share a node, colors run one launch after another,
// and inside a launch every node is written by at most one element. The
// first element to touch a node (in color order) stores its value, later
// elements read-modify-write it; the per-element ownership bitmask built here
// says which of the two each element-local node takes.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "hx_internal.h"

namespace {

uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

struct Centroids {
  std::vector<double> c;  // E*3
  double lo[3], hi[3];
};

Centroids centroids(int P, int64_t E, const int32_t *en, const double *xyz) {
  Centroids C;
  C.c.assign((size_t)E * 3, 0.0);
  const int p = P - 1;
  const int corner[8] = {0, p, p * P, p + p * P, p * P * P, p + p * P * P, p * P + p * P * P,
                         p + p * P + p * P * P};
  for (int d = 0; d < 3; ++d) {
    C.lo[d] = 1e300;
    C.hi[d] = -1e300;
  }
  for (int64_t e = 0; e < E; ++e) {
    for (int v = 0; v < 8; ++v) {
      const int64_t n = en[(size_t)e * P * P * P + corner[v]];
      for (int d = 0; d < 3; ++d) C.c[e * 3 + d] += 0.125 * xyz[n * 3 + d];
    }
    for (int d = 0; d < 3; ++d) {
      C.lo[d] = std::min(C.lo[d], C.c[e * 3 + d]);
      C.hi[d] = std::max(C.hi[d], C.c[e * 3 + d]);
    }
  }
  return C;
}

std::vector<uint64_t> morton_keys(const Centroids &C, int64_t E) {
  std::vector<uint64_t> k(E);
  for (int64_t e = 0; e < E; ++e) {
    uint64_t q[3];
    for (int d = 0; d < 3; ++d) {
      double span = C.hi[d] - C.lo[d];
      double t = span > 0 ? (C.c[e * 3 + d] - C.lo[d]) / span : 0.0;
      q[d] = (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(t * 2097151.0)));
    }
    k[e] = spread3(q[0]) | spread3(q[1]) << 1 | spread3(q[2]) << 2;
  }
  return k;
}

// Greedy distance-1 coloring of the element-node graph in the given visiting order.
int greedy_color(int P3, int64_t nnodes, const int32_t *en, const std::vector<int64_t> &visit,
                 std::vector<int> &color) {
  const int64_t E = (int64_t)visit.size();
  color.assign(E, -1);
  std::vector<uint64_t> used(nnodes, 0);  // colors 0..63 used at each node
  int ncol = 0;
  std::vector<std::vector<uint8_t>> hi_used;  // colors >= 64 (rare), per node, allocated on demand
  for (int64_t t = 0; t < E; ++t) {
    const int64_t e = visit[t];
    const int32_t *nd = en + (size_t)e * P3;
    uint64_t forb = 0;
    for (int l = 0; l < P3; ++l) forb |= used[nd[l]];
    int c;
    if (~forb != 0) {
      c = __builtin_ctzll(~forb);
    } else {
      // slow path: search colors >= 64
      if (hi_used.empty()) hi_used.resize(nnodes);
      c = 64;
      for (;; ++c) {
        bool ok = true;
        for (int l = 0; l < P3 && ok; ++l) {
          const auto &h = hi_used[nd[l]];
          if ((int)h.size() > c - 64 && h[c - 64]) ok = false;
        }
        if (ok) break;
      }
    }
    color[e] = c;
    for (int l = 0; l < P3; ++l) {
      if (c < 64) {
        used[nd[l]] |= 1ULL << c;
      } else {
        auto &h = hi_used[nd[l]];
        if ((int)h.size() <= c - 64) h.resize(c - 63, 0);
        h[c - 64] = 1;
      }
    }
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

// Strips for the strip-scatter collocated kernel (see hx_mesh_s). Element u follows t when u's
// nodes (0, j, k) are t's nodes (p, j, k) for every (j, k): the two share t's r1 = +1 face with
// matching in-face orientation. Chains of followers are cut into strips of at most strip_len(P)
// elements; the strips are colored greedily over the union of their nodes (keeping the fewer
// colors of a Morton and a row visiting order) and ordered like the elements. Inside a strip,
// element w > 0 does not write its r1 = -1 face (element w-1 writes the shared face after adding
// w's part), and ownership follows the strip order. Returns false (no strips) when the chains
// are too short to pay off or the strips need more than 64 colors.
bool build_strips(hx_mesh_s &m, const std::vector<int32_t> &idx, const std::vector<uint64_t> &mk_int,
                  const std::vector<int64_t> &row_key_int, std::vector<int32_t> &selems, std::vector<uint8_t> &glink,
                  std::vector<uint16_t> &sown, std::string &err) {
  const int P = m.P, P2 = P * P, P3 = P2 * P, p = P - 1;
  const int64_t E = m.nelem;
  std::unordered_map<int32_t, std::vector<int32_t>> by_origin;
  by_origin.reserve((size_t)E * 2);
  for (int64_t t = 0; t < E; ++t) by_origin[idx[(size_t)t * P3]].push_back((int32_t)t);
  std::vector<int32_t> nxt(E, -1), prv(E, -1);
  for (int64_t t = 0; t < E; ++t) {
    auto it = by_origin.find(idx[(size_t)t * P3 + p]);
    if (it == by_origin.end()) continue;
    for (int32_t u : it->second) {
      if (u == t || prv[u] != -1) continue;
      bool match = true;
      for (int jk = 0; jk < P2 && match; ++jk)
        match = idx[(size_t)u * P3 + (size_t)jk * P] == idx[(size_t)t * P3 + (size_t)jk * P + p];
      if (match) {
        nxt[t] = u;
        prv[u] = (int32_t)t;
        break;
      }
    }
  }
  std::vector<std::vector<int32_t>> strips;
  std::vector<uint8_t> vis(E, 0);
  auto walk = [&](int32_t t0) {
    std::vector<int32_t> s;
    for (int32_t u = t0; u != -1 && !vis[u]; u = nxt[u]) {
      vis[u] = 1;
      s.push_back(u);
      if ((int)s.size() == hx::strip_len(P)) {
        strips.push_back(s);
        s.clear();
      }
    }
    if (!s.empty()) strips.push_back(s);
  };
  for (int64_t t = 0; t < E; ++t)
    if (prv[t] == -1 && !vis[t]) walk((int32_t)t);
  for (int64_t t = 0; t < E; ++t)  // closed chains (periodic meshes)
    if (!vis[t]) walk((int32_t)t);
  const int64_t S = (int64_t)strips.size();
  if (S * 2 > E) return false;  // mean strip length below 2

  // greedy coloring over the strips' node sets, two visiting orders
  auto key_of = [&](int64_t s) { return strips[s][strips[s].size() / 2]; };
  auto color_strips = [&](const std::vector<int64_t> &visit, std::vector<int> &col) {
    col.assign(S, -1);
    std::vector<uint64_t> used(m.nnodes, 0);
    int ncol = 0;
    for (int64_t s : visit) {
      uint64_t forb = 0;
      for (int32_t el : strips[s])
        for (int l = 0; l < P3; ++l) forb |= used[idx[(size_t)el * P3 + l]];
      if (~forb == 0) return 65;
      const int c = __builtin_ctzll(~forb);
      col[s] = c;
      for (int32_t el : strips[s])
        for (int l = 0; l < P3; ++l) used[idx[(size_t)el * P3 + l]] |= 1ULL << c;
      ncol = std::max(ncol, c + 1);
    }
    return ncol;
  };
  std::vector<int64_t> v1(S), v2(S);
  std::iota(v1.begin(), v1.end(), 0);
  std::iota(v2.begin(), v2.end(), 0);
  std::stable_sort(v1.begin(), v1.end(), [&](int64_t a, int64_t b) { return mk_int[key_of(a)] < mk_int[key_of(b)]; });
  std::stable_sort(v2.begin(), v2.end(), [&](int64_t a, int64_t b) {
    const int64_t *ka = &row_key_int[(size_t)key_of(a) * 3], *kb = &row_key_int[(size_t)key_of(b) * 3];
    for (int d = 2; d >= 0; --d)
      if (ka[d] != kb[d]) return ka[d] < kb[d];
    return false;
  });
  std::vector<int> c1, c2;
  const int n1 = color_strips(v1, c1), n2 = color_strips(v2, c2);
  const std::vector<int> &col = (n2 <= n1) ? c2 : c1;
  const int ncol = std::min(n1, n2);
  if (ncol > 64) return false;
  std::vector<int64_t> ord(S);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    if (col[a] != col[b]) return col[a] < col[b];
    const uint64_t ka = mk_int[key_of(a)], kb = mk_int[key_of(b)];
    return (col[a] & 1) ? ka > kb : ka < kb;
  });
  m.nstrip_colors = ncol;
  m.nstrips = S;
  m.strip_color_start.assign(ncol + 1, 0);
  for (int64_t s = 0; s < S; ++s) m.strip_color_start[col[s] + 1]++;
  for (int c = 0; c < ncol; ++c) m.strip_color_start[c + 1] += m.strip_color_start[c];

  selems.assign((size_t)S * hx::kStrip, -1);
  sown.assign((size_t)E * P2, 0);
  std::vector<uint8_t> seen(m.nnodes, 0);
  std::vector<int32_t> last_color(m.nnodes, -1), last_member(m.nnodes, -1);
  std::vector<int64_t> last_strip(m.nnodes, -1);
  for (int64_t t = 0; t < S; ++t) {
    const auto &st = strips[ord[t]];
    const int c = col[ord[t]];
    for (size_t w = 0; w < st.size(); ++w) {
      const int32_t el = st[w];
      selems[(size_t)t * hx::kStrip + w] = el;
      for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
          for (int i = 0; i < P; ++i) {
            const int32_t n = idx[(size_t)el * P3 + i + P * (j + P * k)];
            if (last_color[n] == c && last_strip[n] != t) {
              err = "strip coloring check failed: two strips of one color share a node";
              return false;
            }
            // inside a strip only consecutive elements share nodes, on their common face
            if (last_strip[n] == t && !(i == 0 && w > 0 && last_member[n] == (int32_t)w - 1)) {
              err = "strip check failed: members other than neighbours share a node";
              return false;
            }
            last_color[n] = c;
            last_strip[n] = t;
            last_member[n] = (int32_t)w;
            if (w > 0 && i == 0) continue;  // written by element w-1
            if (!seen[n]) {
              seen[n] = 1;
              sown[(size_t)el * P2 + j * P + i] |= (uint16_t)(1u << k);
            }
          }
    }
  }

  // Pack whole strips of one color, in the color's order, into groups of at most strip_len(P)
  // elements: one workgroup per group. Where chains are long (lattices) every group is one strip;
  // where they are short (rotated or unstructured elements) a group holds several strips instead
  // of one strip and idle slots. Strips of one color share no node, so the packing changes neither
  // the ownership bits nor the results. Bit w of a group's link byte: slot w + 1 continues the
  // strip of slot w.
  const int SLen = hx::strip_len(P);
  std::vector<int32_t> gel;
  glink.clear();
  std::vector<int64_t> gstart(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) {
    gstart[c] = (int64_t)glink.size();
    int fill = SLen;  // no open group
    for (int64_t t = m.strip_color_start[c]; t < m.strip_color_start[c + 1]; ++t) {
      const int len = (int)strips[ord[t]].size();
      if (fill + len > SLen) {
        gel.insert(gel.end(), hx::kStrip, -1);
        glink.push_back(0);
        fill = 0;
      }
      int32_t *g = gel.data() + (glink.size() - 1) * hx::kStrip;
      for (int w = 0; w < len; ++w) {
        g[fill + w] = selems[(size_t)t * hx::kStrip + w];
        if (w + 1 < len) glink.back() |= (uint8_t)(1u << (fill + w));
      }
      fill += len;
    }
  }
  gstart[ncol] = (int64_t)glink.size();
  selems.swap(gel);
  m.strip_color_start = gstart;
  m.nstrip_groups = (int64_t)glink.size();
  return true;
}

}  // namespace

extern "C" hx_status hx_mesh_nodes_trilinear(int p, int64_t nelem, const int64_t *elem_verts, int64_t nverts,
                                             const double *verts, const int32_t *elem_nodes, int64_t nnodes,
                                             double *node_xyz) {
  if (p < 1 || p > hx::kMaxP - 1) return hx::fail(HX_EINVAL, "p must be in 1..8");
  if (!elem_verts || !verts || !elem_nodes || !node_xyz) return hx::fail(HX_EINVAL, "null pointer");
  if (nelem < 1 || nverts < 1 || nnodes < 1) return hx::fail(HX_EINVAL, "sizes must be positive");
  const int P = p + 1, P3 = P * P * P;
  std::vector<double> x, w;
  hx::gll_nodes_weights(p, x, w);
  std::fill(node_xyz, node_xyz + nnodes * 3, 0.0);
  for (int64_t e = 0; e < nelem; ++e) {
    double V[8][3];
    for (int v = 0; v < 8; ++v) {
      int64_t id = elem_verts[e * 8 + v];
      if (id < 0 || id >= nverts) return hx::fail(HX_ERANGE, "vertex id out of range");
      for (int d = 0; d < 3; ++d) V[v][d] = verts[id * 3 + d];
    }
    for (int k = 0; k < P; ++k)
      for (int j = 0; j < P; ++j)
        for (int i = 0; i < P; ++i) {
          const double r[3] = {x[i], x[j], x[k]};
          double pt[3] = {0, 0, 0};
          for (int v = 0; v < 8; ++v) {
            double N = 1.0;
            for (int d = 0; d < 3; ++d) {
              const int bit = (v >> d) & 1;
              N *= 0.5 * (1.0 + (bit ? r[d] : -r[d]));
            }
            for (int d = 0; d < 3; ++d) pt[d] += N * V[v][d];
          }
          const int64_t n = elem_nodes[e * P3 + i + P * (j + P * k)];
          if (n < 0 || n >= nnodes) return hx::fail(HX_ERANGE, "node id out of range");
          for (int d = 0; d < 3; ++d) node_xyz[n * 3 + d] = pt[d];
        }
  }
  return HX_OK;
}

namespace {

// The mesh builder behind hx_mesh_create (device = true: the arrays go to the current device) and
// hx_mesh_plan (device = false: they stay on the host, and no HIP call is made).
hx_status mesh_build(int p, int64_t nelem, int64_t nnodes, const int32_t *elem_nodes, const double *node_xyz,
                     const uint8_t *dirichlet, bool device, hx_mesh *out) {
  if (!out) return hx::fail(HX_EINVAL, "out is null");
  *out = nullptr;
  if (p < 1 || p > hx::kMaxP - 1) return hx::fail(HX_EINVAL, "p must be in 1..8");
  if (!elem_nodes || !node_xyz) return hx::fail(HX_EINVAL, "elem_nodes and node_xyz must not be null");
  const int P = p + 1, P2 = P * P, P3 = P2 * P;
  if (nelem < 1 || nnodes < 1 || nnodes > INT32_MAX) return hx::fail(HX_EINVAL, "nelem/nnodes out of range");
  if (nelem * (int64_t)P3 >= ((int64_t)1 << 31)) return hx::fail(HX_EINVAL, "nelem*(p+1)^3 must be < 2^31");
  for (int64_t t = 0; t < nelem * P3; ++t)
    if (elem_nodes[t] < 0 || elem_nodes[t] >= nnodes)
      return hx::fail(HX_ERANGE, "elem_nodes entry " + std::to_string(t) + " = " + std::to_string(elem_nodes[t]) +
                                     " outside [0, nnodes)");

  auto *m = new (std::nothrow) hx_mesh_s();
  if (!m) return hx::fail(HX_ENOMEM, "host allocation failed");
  m->p = p;
  m->P = P;
  m->nelem = nelem;
  m->nnodes = nnodes;
  if (device) (void)hipGetDevice(&m->device);
  m->h_xyz.assign(node_xyz, node_xyz + nnodes * 3);

  // coloring: greedy in two visiting orders (Morton of centroids; centroid z-y-x rows),
  // keep the one with fewer colors
  Centroids C = centroids(P, nelem, elem_nodes, node_xyz);
  std::vector<uint64_t> mk = morton_keys(C, nelem);
  std::vector<int64_t> v1(nelem), v2(nelem);
  std::iota(v1.begin(), v1.end(), 0);
  std::iota(v2.begin(), v2.end(), 0);
  std::stable_sort(v1.begin(), v1.end(), [&](int64_t a, int64_t b) { return mk[a] < mk[b]; });
  {
    // rows: quantize each centroid coordinate with a step of about half an element size
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= std::max(C.hi[d] - C.lo[d], 1e-300);
    double h = 0.5 * std::cbrt(vol / (double)nelem);
    std::vector<int64_t> key(nelem * 3);
    for (int64_t e = 0; e < nelem; ++e)
      for (int d = 0; d < 3; ++d) key[e * 3 + d] = (int64_t)std::floor((C.c[e * 3 + d] - C.lo[d]) / h);
    std::stable_sort(v2.begin(), v2.end(), [&](int64_t a, int64_t b) {
      for (int d = 2; d >= 0; --d)
        if (key[a * 3 + d] != key[b * 3 + d]) return key[a * 3 + d] < key[b * 3 + d];
      return false;
    });
  }
  std::vector<int64_t> row_key(nelem * 3);
  {
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= std::max(C.hi[d] - C.lo[d], 1e-300);
    const double h = 0.5 * std::cbrt(vol / (double)nelem);
    for (int64_t e = 0; e < nelem; ++e)
      for (int d = 0; d < 3; ++d) row_key[e * 3 + d] = (int64_t)std::floor((C.c[e * 3 + d] - C.lo[d]) / h);
  }
  std::vector<int> col1, col2;
  int n1 = greedy_color(P3, nnodes, elem_nodes, v1, col1);
  int n2 = greedy_color(P3, nnodes, elem_nodes, v2, col2);
  std::vector<int> &col = (n2 <= n1) ? col2 : col1;
  const int ncol = std::min(n1, n2);
  m->ncolors = ncol;

  // internal order: color-major, Morton order inside a color, reversed on odd colors so each
  // color's launch starts where the previous one ended (its nodes are then still in cache)
  m->order.resize(nelem);
  std::iota(m->order.begin(), m->order.end(), 0);
  std::stable_sort(m->order.begin(), m->order.end(), [&](int32_t a, int32_t b) {
    if (col[a] != col[b]) return col[a] < col[b];
    return (col[a] & 1) ? mk[a] > mk[b] : mk[a] < mk[b];
  });
  m->color_start.assign(ncol + 1, 0);
  for (int64_t e = 0; e < nelem; ++e) m->color_start[col[e] + 1]++;
  for (int c = 0; c < ncol; ++c) m->color_start[c + 1] += m->color_start[c];

  // indices and ownership in internal order
  std::vector<int32_t> idx((size_t)nelem * P3);
  std::vector<uint16_t> own((size_t)nelem * P2, 0);
  std::vector<uint8_t> seen(nnodes, 0);
  for (int64_t t = 0; t < nelem; ++t) {
    const int32_t *src = elem_nodes + (size_t)m->order[t] * P3;
    std::copy(src, src + P3, idx.begin() + (size_t)t * P3);
    for (int k = 0; k < P; ++k)
      for (int ij = 0; ij < P2; ++ij) {
        const int32_t n = src[ij + P2 * k];
        if (!seen[n]) {
          seen[n] = 1;
          own[(size_t)t * P2 + ij] |= (uint16_t)(1u << k);
        }
      }
  }
  m->nuntouched = 0;
  for (int64_t n = 0; n < nnodes; ++n) m->nuntouched += seen[n] ? 0 : 1;

  // sanity: a node appears at most once per color
  {
    std::vector<int32_t> last(nnodes, -1);
    for (int c = 0; c < ncol; ++c)
      for (int64_t t = m->color_start[c]; t < m->color_start[c + 1]; ++t)
        for (int l = 0; l < P3; ++l) {
          const int32_t n = idx[(size_t)t * P3 + l];
          if (last[n] == c) {
            // an element lists the same node twice, or the coloring is wrong
            delete m;
            return hx::fail(HX_EINVAL, "element lists a node more than once, or two elements of one color share a node");
          }
          last[n] = c;
        }
  }

  std::vector<int32_t> af_host;  // affine element numbering {base, s_j, s_k, 0}, empty if not affine
  // compressed restriction: one base id per row along r1 when every row of every element holds
  // consecutive ids (node (i, j, k) = base[j][k] + i); the fused kernels then read P^2 instead of
  // P^3 indices per element
  {
    bool rows = true;
    std::vector<int32_t> rb((size_t)nelem * P2);
    for (int64_t t = 0; t < nelem && rows; ++t)
      for (int r = 0; r < P2 && rows; ++r) {
        const int32_t *row = idx.data() + (size_t)t * P3 + (size_t)r * P;
        for (int i = 1; i < P; ++i)
          if (row[i] != row[0] + i) {
            rows = false;
            break;
          }
        rb[(size_t)t * P2 + r] = row[0];
      }
    if (rows) {
      m->index_mode = 1;
      hipError_t e = device ? m->idx_rows.upload(rb.data(), rb.size()) : hipSuccess;
      if (e != hipSuccess) {
        delete m;
        return hx::hip_fail(e, "mesh upload");
      }
      // affine rows: base[j][k] = base + j s_j + k s_k (a structured numbering inside each element);
      // the kernels then compute every node id from three numbers per element
      bool affine = P > 1;
      std::vector<int32_t> &af = af_host;
      af.assign((size_t)nelem * 4, 0);
      for (int64_t t = 0; t < nelem && affine; ++t) {
        const int32_t *r = rb.data() + (size_t)t * P2;  // [k][j]
        const int64_t b0 = r[0], sj = (int64_t)r[1] - b0, sk = (int64_t)r[P] - b0;
        for (int k = 0; k < P && affine; ++k)
          for (int j = 0; j < P; ++j)
            if ((int64_t)r[k * P + j] != b0 + j * sj + k * sk) {
              affine = false;
              break;
            }
        af[(size_t)t * 4] = (int32_t)b0;
        af[(size_t)t * 4 + 1] = (int32_t)sj;
        af[(size_t)t * 4 + 2] = (int32_t)sk;
      }
      if (!affine) af.clear();
      if (affine) {
        m->index_mode = 2;
        e = device ? m->idx_affine.upload(af.data(), af.size()) : hipSuccess;
        if (e != hipSuccess) {
          delete m;
          return hx::hip_fail(e, "mesh upload");
        }
      }
    }
  }

  // strips for the strip-scatter kernels
  std::vector<int32_t> selems;
  std::vector<uint8_t> glink;
  std::vector<uint16_t> sown;
  bool strips = false;
  if (hx::strip_degree(P)) {
    std::vector<uint64_t> mk_int(nelem);
    std::vector<int64_t> rk_int(nelem * 3);
    for (int64_t t = 0; t < nelem; ++t) {
      mk_int[t] = mk[m->order[t]];
      for (int d = 0; d < 3; ++d) rk_int[t * 3 + d] = row_key[(int64_t)m->order[t] * 3 + d];
    }
    std::string serr;
    strips = build_strips(*m, idx, mk_int, rk_int, selems, glink, sown, serr);
    if (!strips) {
      m->nstrips = 0;
      m->nstrip_groups = 0;
      m->nstrip_colors = 0;
      m->strip_color_start.clear();
    }
  }
  std::vector<uint8_t> fm(nnodes, 1);
  m->nfree = nnodes;
  if (dirichlet) {
    m->nfree = 0;
    for (int64_t n = 0; n < nnodes; ++n) {
      fm[n] = dirichlet[n] ? 0 : 1;
      m->nfree += fm[n];
    }
  }
  if (!device) {
    m->host_only = true;
    m->h_idx = std::move(idx);
    m->h_own = std::move(own);
    if (strips) {
      m->h_strip_elems = std::move(selems);
      m->h_strip_link = std::move(glink);
      m->h_strip_own = std::move(sown);
    }
    *out = m;
    return HX_OK;
  }
  hipError_t e;
  if ((e = m->idx.upload(idx.data(), idx.size())) != hipSuccess ||
      (e = m->own.upload(own.data(), own.size())) != hipSuccess ||
      (e = m->order_d.upload(m->order.data(), m->order.size())) != hipSuccess ||
      (e = m->xyz.upload(node_xyz, (size_t)nnodes * 3)) != hipSuccess ||
      (e = m->freemask.upload(fm.data(), fm.size())) != hipSuccess ||
      (e = m->zeros.upload(std::vector<double>(64, 0.0).data(), 64)) != hipSuccess ||
      (strips && ((e = m->strip_elems.upload(selems.data(), selems.size())) != hipSuccess ||
                  (e = m->strip_link.upload(glink.data(), glink.size())) != hipSuccess ||
                  (e = m->strip_own.upload(sown.data(), sown.size())) != hipSuccess))) {
    delete m;
    return hx::hip_fail(e, "mesh upload");
  }
  *out = m;
  return HX_OK;
}

}  // namespace

extern "C" hx_status hx_mesh_create(int p, int64_t nelem, int64_t nnodes, const int32_t *elem_nodes,
                                    const double *node_xyz, const uint8_t *dirichlet, hx_mesh *out) {
  return mesh_build(p, nelem, nnodes, elem_nodes, node_xyz, dirichlet, true, out);
}

extern "C" hx_status hx_mesh_plan(int p, int64_t nelem, int64_t nnodes, const int32_t *elem_nodes,
                                  const double *node_xyz, const uint8_t *dirichlet, hx_mesh *out) {
  return mesh_build(p, nelem, nnodes, elem_nodes, node_xyz, dirichlet, false, out);
}

extern "C" hx_status hx_mesh_plan_arrays(hx_mesh m, int32_t *idx, uint16_t *own, int32_t *strip_elems,
                                         uint8_t *strip_link, uint16_t *strip_own, int64_t *strip_color_start) {
  if (!m) return hx::fail(HX_EINVAL, "null mesh");
  if (!m->host_only) return hx::fail(HX_EINVAL, "the mesh is not a host-only plan (hx_mesh_plan)");
  if (idx) std::copy(m->h_idx.begin(), m->h_idx.end(), idx);
  if (own) std::copy(m->h_own.begin(), m->h_own.end(), own);
  if (strip_elems) std::copy(m->h_strip_elems.begin(), m->h_strip_elems.end(), strip_elems);
  if (strip_link) std::copy(m->h_strip_link.begin(), m->h_strip_link.end(), strip_link);
  if (strip_own) std::copy(m->h_strip_own.begin(), m->h_strip_own.end(), strip_own);
  if (strip_color_start) std::copy(m->strip_color_start.begin(), m->strip_color_start.end(), strip_color_start);
  return HX_OK;
}

namespace hx {

// Transpose of the element restriction: for every node, the E-vector slots (caller element e, local node
// l) -> e*P^3 + l that hold it, in ascending order (a counting sort over the caller elements), so a
// gather sums a node's contributions in a fixed order.
hx_status mesh_gather_csr(hx_mesh_s &m) {
  if (m.gather_ptr.ptr) return HX_OK;
  const int P3 = m.P * m.P * m.P;
  const int64_t E = m.nelem, n = m.nnodes;
  std::vector<int32_t> idx((size_t)E * P3);
  HX_HIP(hipMemcpy(idx.data(), m.idx.ptr, sizeof(int32_t) * idx.size(), hipMemcpyDeviceToHost));
  std::vector<int32_t> pos_of(E);  // caller element -> internal position
  for (int64_t t = 0; t < E; ++t) pos_of[m.order[t]] = (int32_t)t;
  std::vector<int32_t> ptr(n + 1, 0), slot((size_t)E * P3);
  for (const int32_t nd : idx) ++ptr[nd + 1];
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t ec = 0; ec < E; ++ec) {
    const int32_t *row = idx.data() + (size_t)pos_of[ec] * P3;
    for (int l = 0; l < P3; ++l) slot[fill[row[l]]++] = (int32_t)(ec * P3 + l);
  }
  HX_HIP(m.gather_ptr.upload(ptr.data(), ptr.size()));
  HX_HIP(m.gather_slot.upload(slot.data(), slot.size()));
  return HX_OK;
}

hx_status mesh_slots(hx_mesh_s &m) {
  if (m.slot_ptr.ptr) return HX_OK;
  const int P3 = m.P * m.P * m.P;
  const int64_t E = m.nelem, n = m.nnodes;
  std::vector<int32_t> idx((size_t)E * P3);
  HX_HIP(hipMemcpy(idx.data(), m.idx.ptr, sizeof(int32_t) * idx.size(), hipMemcpyDeviceToHost));
  std::vector<int32_t> ptr(n + 1, 0), slot(idx.size());
  for (const int32_t nd : idx) ++ptr[nd + 1];
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t e = 0; e < E; ++e)
    for (int l = 0; l < P3; ++l) slot[fill[idx[(size_t)e * P3 + l]]++] = (int32_t)(e * P3 + l);
  HX_HIP(m.slot_ptr.upload(ptr.data(), ptr.size()));
  HX_HIP(m.slot_idx.upload(slot.data(), slot.size()));
  return HX_OK;
}

}  // namespace hx

extern "C" hx_status hx_mesh_get_stats(hx_mesh m, hx_mesh_stats *s) {
  if (!m || !s) return hx::fail(HX_EINVAL, "null pointer");
  s->p = m->p;
  s->ncolors = m->ncolors;
  s->nelem = m->nelem;
  s->nnodes = m->nnodes;
  s->nfree = m->nfree;
  s->nuntouched = m->nuntouched;
  s->max_color = 0;
  for (int c = 0; c < m->ncolors; ++c)
    s->max_color = std::max<int64_t>(s->max_color, m->color_start[c + 1] - m->color_start[c]);
  s->nstrips = m->nstrips;
  s->nstrip_colors = m->nstrip_colors;
  s->nstrip_groups = m->nstrip_groups;
  s->index_mode = m->index_mode;
  return HX_OK;
}

extern "C" hx_status hx_mesh_get_order(hx_mesh m, int32_t *order, int64_t *color_start) {
  if (!m) return hx::fail(HX_EINVAL, "null mesh");
  if (order) std::copy(m->order.begin(), m->order.end(), order);
  if (color_start) std::copy(m->color_start.begin(), m->color_start.end(), color_start);
  return HX_OK;
}

extern "C" void hx_mesh_destroy(hx_mesh m) { delete m; }
