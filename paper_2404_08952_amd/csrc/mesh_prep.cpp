// Host-side mesh preparation (see mesh_prep.hpp).
#include "mesh_prep.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <queue>
#include <thread>

namespace dolinc {

namespace {

// Phase timing to stderr when DOLINC_PREP_TIMING is set.
struct PhaseClock {
  bool on = std::getenv("DOLINC_PREP_TIMING") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void lap(const char* what) {
    auto now = std::chrono::steady_clock::now();
    if (on) std::fprintf(stderr, "[prepare] %-22s %8.3f s\n", what, std::chrono::duration<double>(now - t).count());
    t = now;
  }
};

int n_workers() {
  unsigned h = std::thread::hardware_concurrency();
  if (const char* e = std::getenv("DOLINC_PREP_THREADS")) h = (unsigned)std::atoi(e);
  if (h < 1) h = 1;
  if (h > 16) h = 16;
  return (int)h;
}

// Runs fn(begin, end) over [0, n) in contiguous chunks on worker threads.
template <class F>
void parallel_for(int64_t n, F fn) {
  const int T = n < 1024 ? 1 : n_workers();
  if (T == 1) {
    fn((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T);
  for (int t = 0; t < T; ++t) {
    const int64_t a = n * t / T, b = n * (t + 1) / T;
    th.emplace_back([=] { fn(a, b); });
  }
  for (auto& x : th) x.join();
}

struct CellFaces {
  std::vector<int64_t> ptr;   // [n_cells + 1]
  std::vector<int32_t> face;  // face id
  std::vector<uint8_t> side;  // 0 owner, 1 neighbour
};

void build_cell_faces(const dolinc_mesh_desc& d, CellFaces& cf) {
  const int64_t nc = d.n_cells, nf = d.n_faces;
  cf.ptr.assign(nc + 1, 0);
  for (int64_t f = 0; f < nf; ++f) {
    cf.ptr[d.owner[f] + 1]++;
    cf.ptr[d.neighbour[f] + 1]++;
  }
  for (int64_t c = 0; c < nc; ++c) cf.ptr[c + 1] += cf.ptr[c];
  cf.face.resize(2 * nf);
  cf.side.resize(2 * nf);
  std::vector<int64_t> fill(cf.ptr.begin(), cf.ptr.end() - 1);
  // faces are visited in increasing id, so every cell's list is sorted by face id
  for (int64_t f = 0; f < nf; ++f) {
    int64_t a = fill[d.owner[f]]++;
    cf.face[a] = (int32_t)f;
    cf.side[a] = 0;
    int64_t b = fill[d.neighbour[f]]++;
    cf.face[b] = (int32_t)f;
    cf.side[b] = 1;
  }
}

// Skilling's transform of axes to the transposed Hilbert index (J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004), then bit
// interleaving into one key.
uint64_t hilbert_key(uint32_t* X, int n, int b) {
  uint32_t M = 1u << (b - 1);
  for (uint32_t Q = M; Q > 1; Q >>= 1) {
    uint32_t P = Q - 1;
    for (int i = 0; i < n; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  for (int i = 1; i < n; ++i) X[i] ^= X[i - 1];
  uint32_t t = 0;
  for (uint32_t Q = M; Q > 1; Q >>= 1)
    if (X[n - 1] & Q) t ^= Q - 1;
  for (int i = 0; i < n; ++i) X[i] ^= t;
  uint64_t key = 0;
  for (int j = b - 1; j >= 0; --j)
    for (int i = 0; i < n; ++i) key = (key << 1) | ((X[i] >> j) & 1u);
  return key;
}

}  // namespace

void hilbert_order(int dim, int64_t n, const std::vector<double>& pts, std::vector<int32_t>& new_of_old) {
  const int b = dim == 2 ? 31 : 21;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t c = 0; c < n; ++c)
    for (int a = 0; a < dim; ++a) {
      lo[a] = std::min(lo[a], pts[c * dim + a]);
      hi[a] = std::max(hi[a], pts[c * dim + a]);
    }
  double span = 0.0;
  for (int a = 0; a < dim; ++a) span = std::max(span, hi[a] - lo[a]);
  if (span <= 0.0) span = 1.0;
  const double scale = (double)((1u << b) - 1) / span;
  struct KeyIdx {
    uint64_t key;
    int32_t idx;
    bool operator<(const KeyIdx& o) const { return key < o.key || (key == o.key && idx < o.idx); }
  };
  std::vector<KeyIdx> ki(n);
  parallel_for(n, [&](int64_t a0, int64_t a1) {
    for (int64_t c = a0; c < a1; ++c) {
      uint32_t X[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) X[a] = (uint32_t)std::llround((pts[c * dim + a] - lo[a]) * scale);
      ki[c] = KeyIdx{hilbert_key(X, dim, b), (int32_t)c};
    }
  });
  // chunked sort on worker threads, then pairwise merges; (key, index) is
  // a strict total order, so the result does not depend on the split
  const int T = n < 65536 ? 1 : n_workers();
  std::vector<int64_t> bnd(T + 1);
  for (int t = 0; t <= T; ++t) bnd[t] = n * t / T;
  {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) th.emplace_back([&, t] { std::sort(ki.begin() + bnd[t], ki.begin() + bnd[t + 1]); });
    for (auto& x : th) x.join();
  }
  for (int w = 1; w < T; w *= 2) {
    std::vector<std::thread> th;
    for (int t = 0; t + w < T; t += 2 * w) {
      const int64_t a = bnd[t], m = bnd[t + w], e = bnd[std::min(t + 2 * w, T)];
      th.emplace_back([&, a, m, e] { std::inplace_merge(ki.begin() + a, ki.begin() + m, ki.begin() + e); });
    }
    for (auto& x : th) x.join();
  }
  new_of_old.resize(n);
  parallel_for(n, [&](int64_t a0, int64_t a1) {
    for (int64_t i = a0; i < a1; ++i) new_of_old[ki[i].idx] = (int32_t)i;
  });
}

void rcm_order(int64_t n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& adj,
               std::vector<int32_t>& new_of_old) {
  std::vector<int32_t> deg(n);
  for (int64_t i = 0; i < n; ++i) deg[i] = (int32_t)(ptr[i + 1] - ptr[i]);
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int32_t> level(n, -1);
  auto bfs_far = [&](int32_t s) {  // farthest node of least degree from s
    std::vector<int32_t> q{s};
    std::vector<int32_t> touched{s};
    level[s] = 0;
    size_t h = 0;
    int32_t best = s;
    while (h < q.size()) {
      int32_t v = q[h++];
      if (level[v] > level[best] || (level[v] == level[best] && deg[v] < deg[best])) best = v;
      for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k) {
        int32_t w = adj[k];
        if (level[w] < 0 && !seen[w]) {
          level[w] = level[v] + 1;
          q.push_back(w);
          touched.push_back(w);
        }
      }
    }
    for (int32_t v : touched) level[v] = -1;
    return best;
  };
  std::vector<int32_t> byDeg(n);
  std::iota(byDeg.begin(), byDeg.end(), 0);
  std::stable_sort(byDeg.begin(), byDeg.end(), [&](int32_t x, int32_t y) { return deg[x] < deg[y]; });
  std::vector<int32_t> nb;
  for (int32_t s0 : byDeg) {
    if (seen[s0]) continue;
    int32_t s = bfs_far(bfs_far(s0));
    size_t h = order.size();
    order.push_back(s);
    seen[s] = 1;
    while (h < order.size()) {
      int32_t v = order[h++];
      nb.clear();
      for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k)
        if (!seen[adj[k]]) {
          seen[adj[k]] = 1;
          nb.push_back(adj[k]);
        }
      std::stable_sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) { return deg[x] < deg[y]; });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  new_of_old.resize(n);
  for (int64_t i = 0; i < n; ++i) new_of_old[order[n - 1 - i]] = (int32_t)i;
}

dolinc_status extend_desc(const dolinc_mesh_desc& in, ExtendedDesc& X, std::string& msg) {
  X = ExtendedDesc();
  X.d = in;
  X.n_interior = in.n_cells;
  if (!in.face_patch) return DOLINC_OK;
  if (!in.owner || !in.neighbour || !in.neigh_shift) { msg = "null mesh array"; return DOLINC_EINVAL; }
  if (in.n_patches <= 0 || in.n_patches > 1 << 20) { msg = "n_patches must be in [1, 2^20]"; return DOLINC_EINVAL; }
  const int64_t nf = in.n_faces;
  const int dim = in.dim == 2 ? 2 : 3;
  X.nei.assign(in.neighbour, in.neighbour + nf);
  X.shift.assign(in.neigh_shift, in.neigh_shift + nf * dim);
  for (int64_t f = 0; f < nf; ++f) {
    const int32_t p = in.face_patch[f];
    if (in.neighbour[f] == -1) {
      if (p < 0 || p >= in.n_patches) { msg = "boundary face " + std::to_string(f) + " has no valid patch"; return DOLINC_EMESH; }
      X.nei[f] = (int32_t)(in.n_cells + (int64_t)X.bface.size());
      for (int a = 0; a < dim; ++a) X.shift[f * dim + a] = 0.0;
      X.bface.push_back((int32_t)f);
    } else if (p != -1) {
      msg = "face " + std::to_string(f) + " has two cells and a boundary patch";
      return DOLINC_EMESH;
    }
  }
  if (in.n_cells + (int64_t)X.bface.size() >= (int64_t)INT32_MAX) { msg = "mesh too large for 32-bit indices"; return DOLINC_EINVAL; }
  X.d.n_cells = in.n_cells + (int64_t)X.bface.size();
  X.d.neighbour = X.nei.data();
  X.d.neigh_shift = X.shift.data();
  return DOLINC_OK;
}

dolinc_status prepare_mesh(const dolinc_mesh_desc& d, Prepared& P, std::string& msg, int64_t n_interior) {
  if (d.dim != 2 && d.dim != 3) { msg = "dim must be 2 or 3"; return DOLINC_EINVAL; }
  if (d.n_cells <= 0 || d.n_faces <= 0 || d.n_nodes <= 0) { msg = "empty mesh"; return DOLINC_EINVAL; }
  if (d.n_cells >= (int64_t)INT32_MAX || d.n_faces >= (int64_t)INT32_MAX / 2 || d.n_nodes >= (int64_t)INT32_MAX) {
    msg = "mesh too large for 32-bit indices"; return DOLINC_EINVAL;
  }
  if (!d.node_xyz || !d.face_node_ptr || !d.face_nodes || !d.owner || !d.neighbour || !d.neigh_shift) {
    msg = "null mesh array"; return DOLINC_EINVAL;
  }
  if (d.renumber < 0 || d.renumber > 2) { msg = "renumber must be 0, 1 or 2"; return DOLINC_EINVAL; }
  int B = d.part_cells == 0 ? 256 : d.part_cells;
  if (B < 32 || B > 1024) { msg = "part_cells must be in [32, 1024]"; return DOLINC_EINVAL; }
  const int dim = d.dim;
  const int64_t nc = d.n_cells, nf = d.n_faces, nn = d.n_nodes;
  PhaseClock clk;
  if (d.face_node_ptr[0] != 0) { msg = "face_node_ptr[0] must be 0"; return DOLINC_EMESH; }
  for (int64_t f = 0; f < nf; ++f) {
    int64_t m = d.face_node_ptr[f + 1] - d.face_node_ptr[f];
    if ((dim == 2 && m != 2) || (dim == 3 && (m < 3 || m > 64))) {
      msg = "face " + std::to_string(f) + " has " + std::to_string(m) + " nodes";
      return DOLINC_EMESH;
    }
    for (int64_t k = d.face_node_ptr[f]; k < d.face_node_ptr[f + 1]; ++k)
      if (d.face_nodes[k] < 0 || d.face_nodes[k] >= nn) { msg = "face node index out of range"; return DOLINC_EMESH; }
    int32_t o = d.owner[f], n = d.neighbour[f];
    if (o < 0 || o >= nc || n < 0 || n >= nc) { msg = "owner/neighbour out of range at face " + std::to_string(f); return DOLINC_EMESH; }
    if (o == n) { msg = "face " + std::to_string(f) + " joins a cell to itself"; return DOLINC_EMESH; }
    for (int a = 0; a < dim; ++a)
      if (!std::isfinite(d.neigh_shift[f * dim + a])) { msg = "non-finite neighbour shift"; return DOLINC_EMESH; }
  }
  for (int64_t i = 0; i < nn * dim; ++i)
    if (!std::isfinite(d.node_xyz[i])) { msg = "non-finite node coordinate"; return DOLINC_EMESH; }

  clk.lap("validate");
  CellFaces cf;
  build_cell_faces(d, cf);
  clk.lap("cell faces");
  int64_t maxcf = 0;
  const int64_t nint = n_interior < 0 ? nc : n_interior;
  for (int64_t c = 0; c < nc; ++c) {
    int64_t k = cf.ptr[c + 1] - cf.ptr[c];
    if (c < nint && k < dim + 1) {
      msg = "cell " + std::to_string(c) + " is not closed (" + std::to_string(k) + " faces)";
      return DOLINC_EMESH;
    }
    maxcf = std::max(maxcf, k);
  }
  if (maxcf > 255) { msg = "a cell has more than 255 faces"; return DOLINC_EMESH; }

  P = Prepared();
  P.dim = dim; P.n_cells = nc; P.n_faces = nf; P.n_nodes = nn; P.part_cells = B;
  P.n_interior = nint;
  P.max_cell_faces = maxcf;
  if (d.renumber == 0) {
    P.new_of_old.resize(nc);
    std::iota(P.new_of_old.begin(), P.new_of_old.end(), 0);
  } else if (d.renumber == 1) {
    std::vector<int64_t> ptr(cf.ptr);
    std::vector<int32_t> adj(cf.face.size());
    for (int64_t c = 0; c < nc; ++c)
      for (int64_t k = cf.ptr[c]; k < cf.ptr[c + 1]; ++k) {
        int32_t f = cf.face[k];
        adj[k] = cf.side[k] == 0 ? d.neighbour[f] : d.owner[f];
      }
    rcm_order(nc, ptr, adj, P.new_of_old);
  } else {
    // cell position estimate: mean of its faces' vertex averages (own frame)
    std::vector<double> fc(nf * dim, 0.0);
    parallel_for(nf, [&](int64_t f0, int64_t f1) {
      for (int64_t f = f0; f < f1; ++f) {
        int64_t a = d.face_node_ptr[f], b = d.face_node_ptr[f + 1];
        for (int64_t k = a; k < b; ++k)
          for (int ax = 0; ax < dim; ++ax) fc[f * dim + ax] += d.node_xyz[(int64_t)d.face_nodes[k] * dim + ax];
        for (int ax = 0; ax < dim; ++ax) fc[f * dim + ax] /= (double)(b - a);
      }
    });
    std::vector<double> pts(nc * dim, 0.0);
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
      for (int64_t c = c0; c < c1; ++c) {
        for (int64_t k = cf.ptr[c]; k < cf.ptr[c + 1]; ++k) {
          int32_t f = cf.face[k];
          for (int ax = 0; ax < dim; ++ax)
            pts[c * dim + ax] += fc[f * dim + ax] - (cf.side[k] ? d.neigh_shift[f * dim + ax] : 0.0);
        }
        for (int ax = 0; ax < dim; ++ax) pts[c * dim + ax] /= (double)(cf.ptr[c + 1] - cf.ptr[c]);
      }
    });
    hilbert_order(dim, nc, pts, P.new_of_old);
  }
  if (nint < nc) {
    // auxiliary cells keep their rows after the renumbered interior cells
    std::vector<int32_t> order(nc), nn2(nc);
    for (int64_t c = 0; c < nc; ++c) order[P.new_of_old[c]] = (int32_t)c;
    int32_t next = 0;
    for (int64_t i = 0; i < nc; ++i)
      if (order[i] < nint) nn2[order[i]] = next++;
    for (int64_t c = nint; c < nc; ++c) nn2[c] = (int32_t)c;
    P.new_of_old.swap(nn2);
  }
  clk.lap("renumber");
  P.old_of_new.resize(nc);
  for (int64_t c = 0; c < nc; ++c) P.old_of_new[P.new_of_old[c]] = (int32_t)c;

  // partitions, entries, slots: every partition is built independently
  // (its faces in order of first touch by its cells, cells in order, each
  // cell's faces by id) and the pieces are concatenated in partition order
  P.n_parts = (nc + B - 1) / B;
  P.part_ent_ptr.assign(P.n_parts + 1, 0);
  P.slot_ptr.assign(nc + 1, 0);
  P.slots.resize(2 * nf);
  P.face_first_ent.assign(nf, -1);
  std::vector<std::vector<int32_t>> pfaces(P.n_parts);
  std::vector<int64_t> maxloc(P.n_parts, 0);
  bool too_many = false;
  parallel_for(P.n_parts, [&](int64_t p0, int64_t p1) {
    std::vector<std::pair<int32_t, int32_t>> seen;  // (face, first-touch order)
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t c0 = p * B, c1 = std::min<int64_t>(c0 + B, nc);
      seen.clear();
      for (int64_t c = c0; c < c1; ++c) {
        const int32_t oc = P.old_of_new[c];
        for (int64_t k = cf.ptr[oc]; k < cf.ptr[oc + 1]; ++k) seen.emplace_back(cf.face[k], (int32_t)seen.size());
      }
      std::sort(seen.begin(), seen.end());
      // keep the first touch of every face; order the faces by first touch
      std::vector<std::pair<int32_t, int32_t>> firsts;  // (first touch, face)
      for (size_t i = 0; i < seen.size(); ++i)
        if (i == 0 || seen[i].first != seen[i - 1].first) firsts.emplace_back(seen[i].second, seen[i].first);
      std::sort(firsts.begin(), firsts.end());
      std::vector<int32_t>& fl = pfaces[p];
      fl.resize(firsts.size());
      for (size_t i = 0; i < firsts.size(); ++i) fl[i] = firsts[i].second;
      maxloc[p] = (int64_t)fl.size();
      if (fl.size() >= 32768) too_many = true;
      for (int64_t c = c0; c < c1; ++c) {
        const int32_t oc = P.old_of_new[c];
        P.slot_ptr[c + 1] = (int32_t)(cf.ptr[oc + 1] - cf.ptr[oc]);
      }
    }
  });
  if (too_many) { msg = "partition has too many faces"; return DOLINC_EMESH; }
  for (int64_t c = 0; c < nc; ++c) P.slot_ptr[c + 1] += P.slot_ptr[c];
  for (int64_t p = 0; p < P.n_parts; ++p) {
    P.part_ent_ptr[p + 1] = P.part_ent_ptr[p] + (int32_t)pfaces[p].size();
    P.max_entries = std::max(P.max_entries, maxloc[p]);
  }
  if ((int64_t)P.part_ent_ptr[P.n_parts] >= (int64_t)INT32_MAX / 2) { msg = "too many face entries"; return DOLINC_EMESH; }
  const int64_t ne = P.part_ent_ptr[P.n_parts];
  P.ent_face.resize(ne);
  P.ent_p.resize(ne);
  P.ent_n.resize(ne);
  parallel_for(P.n_parts, [&](int64_t p0, int64_t p1) {
    std::vector<std::pair<int32_t, int32_t>> byface;
    for (int64_t p = p0; p < p1; ++p) {
      const std::vector<int32_t>& fl = pfaces[p];
      const int64_t e0 = P.part_ent_ptr[p];
      byface.resize(fl.size());
      for (size_t i = 0; i < fl.size(); ++i) {
        const int32_t f = fl[i];
        P.ent_face[e0 + i] = f;
        P.ent_p[e0 + i] = P.new_of_old[d.owner[f]];
        P.ent_n[e0 + i] = P.new_of_old[d.neighbour[f]];
        byface[i] = std::make_pair(f, (int32_t)i);
      }
      std::sort(byface.begin(), byface.end());
      const int64_t c0 = p * B, c1 = std::min<int64_t>(c0 + B, nc);
      for (int64_t c = c0; c < c1; ++c) {
        const int32_t oc = P.old_of_new[c];
        int64_t s = P.slot_ptr[c];
        for (int64_t k = cf.ptr[oc]; k < cf.ptr[oc + 1]; ++k) {
          const int32_t f = cf.face[k];
          auto it = std::lower_bound(byface.begin(), byface.end(), std::make_pair(f, (int32_t)-1));
          P.slots[s++] = (uint16_t)(it->second | (cf.side[k] << 15));
        }
      }
    }
  });
  // first entry of every face (lowest partition wins)
  for (int64_t e = ne - 1; e >= 0; --e) P.face_first_ent[P.ent_face[e]] = (int32_t)e;
  // a seam face has a second entry; every slot names the other one
  {
    std::vector<int32_t> second(nf, -1);
    for (int64_t e = 0; e < ne; ++e)
      if (P.face_first_ent[P.ent_face[e]] != (int32_t)e) second[P.ent_face[e]] = (int32_t)e;
    P.slot_twin.assign(P.slots.size(), -1);
    parallel_for(P.n_parts, [&](int64_t p0, int64_t p1) {
      for (int64_t p = p0; p < p1; ++p) {
        const int64_t e0 = P.part_ent_ptr[p];
        const int64_t c0 = p * B, c1 = std::min<int64_t>(c0 + B, nc);
        for (int64_t s = P.slot_ptr[c0]; s < P.slot_ptr[c1]; ++s) {
          const int64_t e = e0 + (P.slots[s] & 0x7fff);
          const int32_t f = P.ent_face[e];
          const int32_t o = P.face_first_ent[f] == (int32_t)e ? second[f] : P.face_first_ent[f];
          P.slot_twin[s] = o < 0 ? -1 : 2 * o + (P.slots[s] >> 15);
        }
      }
    });
  }
  clk.lap("partitions");
  if ((int64_t)P.ent_face.size() >= (int64_t)INT32_MAX) { msg = "too many face entries"; return DOLINC_EMESH; }
  return DOLINC_OK;
}

}  // namespace dolinc
