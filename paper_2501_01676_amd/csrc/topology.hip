// Host-side box-partition topology (see topology.h).
#include "topology.h"

#include <algorithm>
#include <array>

#include "host_pool.h"
#include "htrace.h"
#include "internal.h"

namespace abddc {

int SubInfo::local_pos(int obj) const {
  auto it = std::lower_bound(objs.begin(), objs.end(), obj);
  if (it == objs.end() || *it != obj) return -1;
  return obj_off[it - objs.begin()];
}

void Topology::build_grid(const int nsub_in[3], const int* const width_in[3]) {
  for (int a = 0; a < 3; ++a) {
    nsub[a] = nsub_in[a];
    ABDDC_REQUIRE(nsub[a] >= 1, ABDDC_EINVAL, "nsub must be >= 1");
    widths[a].assign(width_in[a], width_in[a] + nsub[a]);
    cuts[a].assign(1, 0);
    for (int w : widths[a]) {
      ABDDC_REQUIRE(w >= 2, ABDDC_EINVAL, "every subdomain width must be >= 2 elements");
      cuts[a].push_back(cuts[a].back() + w);
    }
    ne[a] = cuts[a].back();
    nn[a] = ne[a] + 1;
  }
  n_sub = nsub[0] * nsub[1] * nsub[2];
  n_nodes = (int64_t)nn[0] * nn[1] * nn[2];
  n_elem = (int64_t)ne[0] * ne[1] * ne[2];
}

void Topology::build(const int nsub_in[3], const int* const width_in[3]) {
  build_grid(nsub_in, width_in);
  build_objects();
}

void Topology::build_objects() {
  HostTrace ht;
  // Per axis, a grid index has the key 2s inside subdomain s and 2c - 1 on
  // the cut c between subdomains c - 1 and c; the indices of one key form
  // the range [klo, khi] (Dirichlet boundary indices belong to no key).  An
  // interface object is a key triple with at least one odd key, its nodes
  // the tensor product of the three ranges, its subdomains those holding
  // every one of them; one odd key makes a face, two an edge, three a vertex.
  std::vector<int> klo[3], khi[3];
  for (int a = 0; a < 3; ++a) {
    const int nk = 2 * nsub[a] - 1;
    klo[a].assign(nk, 0);
    khi[a].assign(nk, 0);
    for (int s = 0; s < nsub[a]; ++s) {
      klo[a][2 * s] = cuts[a][s] + 1;
      khi[a][2 * s] = cuts[a][s + 1] - 1;
    }
    for (int c = 1; c < nsub[a]; ++c) klo[a][2 * c - 1] = khi[a][2 * c - 1] = cuts[a][c];
  }
  // free nodes: the grid minus its boundary, numbered by node id (dof_of)
  n_dof = (int64_t)(nn[0] - 2) * (nn[1] - 2) * (nn[2] - 2);
  objects.clear();
  const int nk[3] = {2 * nsub[0] - 1, 2 * nsub[1] - 1, 2 * nsub[2] - 1};
  // key triples in interface order: faces, edges, vertices, each by their
  // first node id, which grows with (kz, ky, kx) lexicographically because
  // every range's lower end grows with its key
  std::vector<std::array<int, 3>> keys;
  for (int odd = 1; odd <= 3; ++odd)
    for (int kz = 0; kz < nk[2]; ++kz)
      for (int ky = 0; ky < nk[1]; ++ky)
        for (int kx = 0; kx < nk[0]; ++kx)
          if ((kx & 1) + (ky & 1) + (kz & 1) == odd) keys.push_back({kx, ky, kz});
  objects.resize(keys.size());
  host_parallel_for((int64_t)keys.size(), 64, [&](int64_t b, int64_t e) {
    for (int64_t q = b; q < e; ++q) {
      const int* key = keys[q].data();
      const int odd = (key[0] & 1) + (key[1] & 1) + (key[2] & 1);
      Object& o = objects[q];
      o.kind = odd == 1 ? KIND_FACE : (odd == 2 ? KIND_EDGE : KIND_VERTEX);
      int slo[3], shi[3];
      for (int a = 0; a < 3; ++a) {
        o.lo[a] = klo[a][key[a]];
        o.hi[a] = khi[a][key[a]];
        slo[a] = key[a] / 2;
        shi[a] = (key[a] + 1) / 2;
      }
      for (int sz = slo[2]; sz <= shi[2]; ++sz)
        for (int sy = slo[1]; sy <= shi[1]; ++sy)
          for (int sx = slo[0]; sx <= shi[0]; ++sx) o.subs.push_back(sub_id(sx, sy, sz));
      std::sort(o.subs.begin(), o.subs.end());
      o.nodes.reserve((size_t)(o.hi[0] - o.lo[0] + 1) * (o.hi[1] - o.lo[1] + 1) * (o.hi[2] - o.lo[2] + 1));
      for (int iz = o.lo[2]; iz <= o.hi[2]; ++iz)
        for (int iy = o.lo[1]; iy <= o.hi[1]; ++iy)
          for (int ix = o.lo[0]; ix <= o.hi[0]; ++ix) o.nodes.push_back(node_id(ix, iy, iz));
      o.n = (int)o.nodes.size();
    }
  });

  ht.mark("topology: objects");
  faces.clear();
  edges.clear();
  vertices.clear();
  kind_index.assign(objects.size(), 0);
  int64_t g = 0;
  for (size_t k = 0; k < objects.size(); ++k) {
    Object& o = objects[k];
    o.gstart = g;
    g += o.n;
    std::vector<int>& lst = o.kind == KIND_FACE ? faces : (o.kind == KIND_EDGE ? edges : vertices);
    kind_index[k] = (int)lst.size();
    lst.push_back((int)k);
  }
  n_gamma = g;

  // object of each key triple (-1: no object)
  std::vector<int> obj_of_key((size_t)nk[0] * nk[1] * nk[2], -1);
  for (size_t q = 0; q < keys.size(); ++q)
    obj_of_key[keys[q][0] + (size_t)nk[0] * (keys[q][1] + (size_t)nk[1] * keys[q][2])] = (int)q;
  sub.assign(n_sub, SubInfo());
  ht.mark("topology: interface numbering");
  host_parallel_for(n_sub, 8, [&](int64_t b, int64_t e) {
    for (int s = (int)b; s < (int)e; ++s) {
      const int sx = s % nsub[0], sy = (s / nsub[0]) % nsub[1], sz = s / (nsub[0] * nsub[1]);
      const int sc[3] = {sx, sy, sz};
      SubInfo& si = sub[s];
      // the objects of subdomain s: the key triples with every key in
      // {2 s_a - 1, 2 s_a, 2 s_a + 1}, in interface order
      for (int kz = 2 * sz - 1; kz <= 2 * sz + 1; ++kz)
        for (int ky = 2 * sy - 1; ky <= 2 * sy + 1; ++ky)
          for (int kx = 2 * sx - 1; kx <= 2 * sx + 1; ++kx) {
            if (kx < 0 || ky < 0 || kz < 0 || kx >= nk[0] || ky >= nk[1] || kz >= nk[2]) continue;
            const int q = obj_of_key[kx + (size_t)nk[0] * (ky + (size_t)nk[1] * kz)];
            if (q >= 0) si.objs.push_back(q);
          }
      std::sort(si.objs.begin(), si.objs.end());
      for (int a = 0; a < 3; ++a) {
        si.ebox[a][0] = cuts[a][sc[a]];
        si.ebox[a][1] = cuts[a][sc[a] + 1];
      }
      si.interior.reserve((size_t)(si.ebox[0][1] - si.ebox[0][0] - 1) * (si.ebox[1][1] - si.ebox[1][0] - 1) *
                          (si.ebox[2][1] - si.ebox[2][0] - 1));
      for (int iz = si.ebox[2][0] + 1; iz < si.ebox[2][1]; ++iz)
        for (int iy = si.ebox[1][0] + 1; iy < si.ebox[1][1]; ++iy)
          for (int ix = si.ebox[0][0] + 1; ix < si.ebox[0][1]; ++ix) si.interior.push_back(node_id(ix, iy, iz));
      si.nI = (int)si.interior.size();
      int pos = 0;
      for (int k : si.objs) pos += objects[k].n;
      si.gamma.reserve(pos);
      pos = 0;
      for (int k : si.objs) {
        si.obj_off.push_back(pos);
        for (int q = 0; q < objects[k].n; ++q) si.gamma.push_back(objects[k].gstart + q);
        pos += objects[k].n;
      }
      si.nB = pos;
    }
  });
  ht.mark("topology: subdomain lists");
}

}  // namespace abddc

namespace abddc {

void Topology::build_partition(const int32_t* part, int n_parts) {
  ABDDC_REQUIRE(nsub[0] == 1 && nsub[1] == 1 && nsub[2] == 1, ABDDC_EINVAL,
                "a general partition takes the grid as one subdomain per axis");
  ABDDC_REQUIRE(n_parts >= 1, ABDDC_EINVAL, "n_parts must be >= 1");
  general = true;
  n_sub = n_parts;
  std::vector<int64_t> boxes_of(n_parts, 0);
  for (int64_t e = 0; e < n_elem; ++e) {
    ABDDC_REQUIRE(part[e] >= 0 && part[e] < n_parts, ABDDC_EINVAL, "part id outside [0, n_parts)");
    ++boxes_of[part[e]];
  }
  for (int p = 0; p < n_parts; ++p) ABDDC_REQUIRE(boxes_of[p] > 0, ABDDC_EINVAL, "a part holds no box");
  n_dof = (int64_t)(nn[0] - 2) * (nn[1] - 2) * (nn[2] - 2);
  // sharing set of every free node: the sorted distinct parts of its boxes
  std::vector<std::array<int, 8>> sets(n_nodes);
  std::vector<uint8_t> nset(n_nodes, 0);
  for (int64_t v = 0; v < n_nodes; ++v) {
    if (dof_of(v) < 0) continue;
    const int ix = (int)(v % nn[0]), iy = (int)((v / nn[0]) % nn[1]), iz = (int)(v / ((int64_t)nn[0] * nn[1]));
    std::array<int, 8>& S = sets[v];
    int k = 0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int bx = ix - dx, by = iy - dy, bz = iz - dz;   // free nodes have all 8 boxes
          S[k++] = part[bx + (int64_t)ne[0] * (by + (int64_t)ne[1] * bz)];
        }
    std::sort(S.begin(), S.end());
    nset[v] = (uint8_t)(std::unique(S.begin(), S.end()) - S.begin());
  }
  auto same_set = [&](int64_t a, int64_t b) {
    if (nset[a] != nset[b]) return false;
    for (int i = 0; i < nset[a]; ++i)
      if (sets[a][i] != sets[b][i]) return false;
    return true;
  };
  // connected pieces of equal sharing sets (26-neighbourhood), found from
  // each piece's smallest node, so the pieces come out by first node
  objects.clear();
  std::vector<char> seen(n_nodes, 0);
  std::vector<int64_t> stack;
  for (int64_t v0 = 0; v0 < n_nodes; ++v0) {
    if (nset[v0] < 2 || seen[v0]) continue;   // Dirichlet nodes have no set
    Object o;
    o.subs.assign(sets[v0].begin(), sets[v0].begin() + nset[v0]);
    stack.assign(1, v0);
    seen[v0] = 1;
    while (!stack.empty()) {
      const int64_t v = stack.back();
      stack.pop_back();
      o.nodes.push_back(v);
      const int ix = (int)(v % nn[0]), iy = (int)((v / nn[0]) % nn[1]), iz = (int)(v / ((int64_t)nn[0] * nn[1]));
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int qx = ix + dx, qy = iy + dy, qz = iz + dz;
            if (qx < 0 || qy < 0 || qz < 0 || qx >= nn[0] || qy >= nn[1] || qz >= nn[2]) continue;
            const int64_t w = node_id(qx, qy, qz);
            if (seen[w] || nset[w] == 0 || !same_set(v0, w)) continue;
            seen[w] = 1;
            stack.push_back(w);
          }
    }
    std::sort(o.nodes.begin(), o.nodes.end());
    o.n = (int)o.nodes.size();
    o.kind = o.subs.size() == 2 ? KIND_FACE : (o.n >= 2 ? KIND_EDGE : KIND_VERTEX);
    for (int a = 0; a < 3; ++a) {
      o.lo[a] = nn[a];
      o.hi[a] = -1;
    }
    for (int64_t v : o.nodes) {
      const int c[3] = {(int)(v % nn[0]), (int)((v / nn[0]) % nn[1]), (int)(v / ((int64_t)nn[0] * nn[1]))};
      for (int a = 0; a < 3; ++a) {
        o.lo[a] = std::min(o.lo[a], c[a]);
        o.hi[a] = std::max(o.hi[a], c[a]);
      }
    }
    objects.push_back(std::move(o));
  }
  std::stable_sort(objects.begin(), objects.end(),
                   [](const Object& a, const Object& b) { return a.kind < b.kind; });
  faces.clear();
  edges.clear();
  vertices.clear();
  kind_index.assign(objects.size(), 0);
  int64_t g = 0;
  for (size_t k = 0; k < objects.size(); ++k) {
    Object& o = objects[k];
    o.gstart = g;
    g += o.n;
    std::vector<int>& lst = o.kind == KIND_FACE ? faces : (o.kind == KIND_EDGE ? edges : vertices);
    kind_index[k] = (int)lst.size();
    lst.push_back((int)k);
  }
  n_gamma = g;
  sub.assign(n_sub, SubInfo());
  for (int s = 0; s < n_sub; ++s)
    for (int a = 0; a < 3; ++a) {
      sub[s].ebox[a][0] = ne[a];
      sub[s].ebox[a][1] = 0;
    }
  for (int64_t e = 0; e < n_elem; ++e) {
    const int c[3] = {(int)(e % ne[0]), (int)((e / ne[0]) % ne[1]), (int)(e / ((int64_t)ne[0] * ne[1]))};
    SubInfo& si = sub[part[e]];
    for (int a = 0; a < 3; ++a) {
      si.ebox[a][0] = std::min(si.ebox[a][0], c[a]);
      si.ebox[a][1] = std::max(si.ebox[a][1], c[a] + 1);
    }
  }
  for (int64_t v = 0; v < n_nodes; ++v)
    if (nset[v] == 1) sub[sets[v][0]].interior.push_back(v);   // (0 for Dirichlet nodes)
  for (size_t k = 0; k < objects.size(); ++k)
    for (int s : objects[k].subs) sub[s].objs.push_back((int)k);
  for (int s = 0; s < n_sub; ++s) {
    SubInfo& si = sub[s];
    si.nI = (int)si.interior.size();
    int pos = 0;
    for (int k : si.objs) {
      si.obj_off.push_back(pos);
      for (int q = 0; q < objects[k].n; ++q) si.gamma.push_back(objects[k].gstart + q);
      pos += objects[k].n;
    }
    si.nB = pos;
  }
}

}  // namespace abddc
