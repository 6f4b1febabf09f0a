// Host-side box-partition topology (see topology.h).
#include "topology.h"

#include <algorithm>

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
  // per-axis: is grid index on an internal cut, and which subdomains hold it
  std::vector<char> oncut[3];
  std::vector<int> s_lo[3], s_hi[3];
  for (int a = 0; a < 3; ++a) {
    oncut[a].assign(nn[a], 0);
    s_lo[a].assign(nn[a], 0);
    s_hi[a].assign(nn[a], 0);
    for (int c = 1; c < nsub[a]; ++c) oncut[a][cuts[a][c]] = 1;
    for (int i = 0; i < nn[a]; ++i) {
      int lo = -1, hi = -1;
      for (int s = 0; s < nsub[a]; ++s)
        if (cuts[a][s] <= i && i <= cuts[a][s + 1]) {
          if (lo < 0) lo = s;
          hi = s;
        }
      s_lo[a][i] = lo;
      s_hi[a][i] = hi;
    }
  }

  dof_of_node.assign(n_nodes, -1);
  iface_of_node.assign(n_nodes, -1);
  // The sharing set of a node is fixed by (s_lo + s_hi) per axis: 2s inside
  // subdomain s, 2s + 1 on the cut between s and s + 1; those three numbers
  // index a dense table of objects.
  const int kx = 2 * nsub[0] - 1, ky = 2 * nsub[1] - 1, kz = 2 * nsub[2] - 1;
  std::vector<int> obj_of_key((size_t)kx * ky * kz, -1);
  objects.clear();
  int64_t ndof = 0;
  for (int iz = 0; iz < nn[2]; ++iz)
    for (int iy = 0; iy < nn[1]; ++iy)
      for (int ix = 0; ix < nn[0]; ++ix) {
        const int64_t nid = node_id(ix, iy, iz);
        const bool fr = ix > 0 && ix < nn[0] - 1 && iy > 0 && iy < nn[1] - 1 && iz > 0 && iz < nn[2] - 1;
        if (!fr) continue;
        dof_of_node[nid] = ndof++;
        const int cnt = oncut[0][ix] + oncut[1][iy] + oncut[2][iz];
        if (cnt == 0) continue;
        const size_t key = (size_t)(s_lo[0][ix] + s_hi[0][ix]) +
                           (size_t)kx * ((s_lo[1][iy] + s_hi[1][iy]) + (size_t)ky * (s_lo[2][iz] + s_hi[2][iz]));
        int k = obj_of_key[key];
        if (k < 0) {
          Object o;
          for (int sz = s_lo[2][iz]; sz <= s_hi[2][iz]; ++sz)
            for (int sy = s_lo[1][iy]; sy <= s_hi[1][iy]; ++sy)
              for (int sx = s_lo[0][ix]; sx <= s_hi[0][ix]; ++sx) o.subs.push_back(sub_id(sx, sy, sz));
          std::sort(o.subs.begin(), o.subs.end());
          ABDDC_REQUIRE(o.subs.size() == 2 || o.subs.size() == 4 || o.subs.size() == 8, ABDDC_EINVAL,
                        "unexpected interface class");
          o.kind = o.subs.size() == 2 ? KIND_FACE : (o.subs.size() == 4 ? KIND_EDGE : KIND_VERTEX);
          k = (int)objects.size();
          obj_of_key[key] = k;
          objects.push_back(std::move(o));
        }
        objects[k].nodes.push_back(nid);   // visited in increasing node id
      }
  n_dof = ndof;
  for (Object& o : objects) o.n = (int)o.nodes.size();
  std::sort(objects.begin(), objects.end(), [](const Object& a, const Object& b) {
    if (a.kind != b.kind) return a.kind < b.kind;
    return a.nodes[0] < b.nodes[0];
  });
  faces.clear();
  edges.clear();
  vertices.clear();
  kind_index.assign(objects.size(), 0);
  int64_t g = 0;
  for (size_t k = 0; k < objects.size(); ++k) {
    Object& o = objects[k];
    o.gstart = g;
    for (int q = 0; q < o.n; ++q) iface_of_node[o.nodes[q]] = g + q;
    g += o.n;
    std::vector<int>& lst = o.kind == KIND_FACE ? faces : (o.kind == KIND_EDGE ? edges : vertices);
    kind_index[k] = (int)lst.size();
    lst.push_back((int)k);
  }
  n_gamma = g;

  sub.assign(n_sub, SubInfo());
  for (int s = 0; s < n_sub; ++s) {
    const int sx = s % nsub[0], sy = (s / nsub[0]) % nsub[1], sz = s / (nsub[0] * nsub[1]);
    const int sc[3] = {sx, sy, sz};
    SubInfo& si = sub[s];
    for (int a = 0; a < 3; ++a) {
      si.ebox[a][0] = cuts[a][sc[a]];
      si.ebox[a][1] = cuts[a][sc[a] + 1];
    }
    for (int iz = si.ebox[2][0] + 1; iz < si.ebox[2][1]; ++iz)
      for (int iy = si.ebox[1][0] + 1; iy < si.ebox[1][1]; ++iy)
        for (int ix = si.ebox[0][0] + 1; ix < si.ebox[0][1]; ++ix) si.interior.push_back(node_id(ix, iy, iz));
    si.nI = (int)si.interior.size();
  }
  for (size_t k = 0; k < objects.size(); ++k)
    for (int s : objects[k].subs) sub[s].objs.push_back((int)k);
  for (int s = 0; s < n_sub; ++s) {
    SubInfo& si = sub[s];
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
