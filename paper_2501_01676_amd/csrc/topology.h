// Host-side partition topology: interface classes and orderings.
//
// Box partitions: a free grid node on an internal subdomain cut plane in
// exactly one / two / three axes is a face / edge / vertex node; nodes with
// the same set n(x) of sharing subdomains form one interface object.
// General partitions (every subdomain a union of grid boxes): n(x) = the
// subdomains holding a box incident to the free node x; |n(x)| = 1 makes x
// interior; the nodes with one sharing set split into connected pieces (two
// nodes adjacent when a box holds both), each piece one object: a face when
// |n(x)| = 2, an edge when |n(x)| >= 3 and the piece has two or more nodes,
// else a vertex.  (Section 3 defers the definitions of faces, edges and
// vertices; these are the rules read here.)  Orderings are part of the C ABI
// (include/abddc.h).
#pragma once

#include <cstdint>
#include <vector>

namespace abddc {

enum ObjKind { KIND_FACE = 0, KIND_EDGE = 1, KIND_VERTEX = 2 };

struct Object {
  int kind;
  std::vector<int> subs;        // sorted subdomain ids n(X)
  std::vector<int64_t> nodes;   // sorted grid node ids
  int64_t gstart;               // first interface index
  int n;                        // number of dofs
  int lo[3], hi[3];             // grid index box [lo, hi] (inclusive) per axis holding the nodes
                                // (exactly the nodes on box partitions)
};

struct SubInfo {
  int ebox[3][2];               // element index range [lo, hi) per axis (the subdomain's
                                // bounding box on general partitions)
  std::vector<int64_t> interior;  // grid node ids, sorted
  std::vector<int64_t> gamma;     // interface indices, sorted
  std::vector<int> objs;          // objects of Gamma_i, interface order
  std::vector<int> obj_off;       // local offset of each object inside Gamma_i
  int nI = 0, nB = 0;
  int local_pos(int obj) const;   // offset of object obj in Gamma_i or -1
};

struct Topology {
  int nsub[3];
  std::vector<int> widths[3];
  std::vector<int> cuts[3];
  int ne[3], nn[3];
  int64_t n_nodes, n_elem, n_dof, n_gamma;
  int n_sub;
  std::vector<Object> objects;
  std::vector<int> faces, edges, vertices;   // indices into objects
  std::vector<int> kind_index;               // position of object within its kind
  std::vector<SubInfo> sub;

  void build(const int nsub_in[3], const int* const width_in[3]);
  // the two halves of build: the grid (cuts, sizes), then the interface
  // objects and subdomain lists
  void build_grid(const int nsub_in[3], const int* const width_in[3]);
  void build_objects();
  // general partition: part[box] in [0, n_parts) per box (x-fastest), each
  // part non-empty; after build_grid with one subdomain per axis
  void build_partition(const int32_t* part, int n_parts);
  bool general = false;         // built by build_partition
  int64_t node_id(int64_t ix, int64_t iy, int64_t iz) const { return ix + nn[0] * (iy + (int64_t)nn[1] * iz); }
  // global dof of node v: the free nodes (the grid minus its boundary)
  // numbered by node id; -1 for a Dirichlet node
  int64_t dof_of(int64_t v) const {
    const int64_t ix = v % nn[0], iy = (v / nn[0]) % nn[1], iz = v / ((int64_t)nn[0] * nn[1]);
    if (ix == 0 || iy == 0 || iz == 0 || ix == nn[0] - 1 || iy == nn[1] - 1 || iz == nn[2] - 1) return -1;
    return (ix - 1) + (int64_t)(nn[0] - 2) * ((iy - 1) + (int64_t)(nn[1] - 2) * (iz - 1));
  }
  int sub_id(int sx, int sy, int sz) const { return sx + nsub[0] * (sy + nsub[1] * sz); }
};

}  // namespace abddc
