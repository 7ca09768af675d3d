// Host runtime for meshes beyond the lattice of trilinear cells: general hexahedral meshes given
// by connectivity (node numbering, gather map, node -> slot lists, constraints), curved cells given
// by their map at equispaced points (stored geometry per quadrature point), and the host-side
// geometry queries (node positions, pressure loads) for every kind of context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "hx.h"
#include "hx_context.hpp"
#include "hx_internal.hpp"

namespace hx {
namespace {

// Lagrange basis on the g+1 equispaced points i/g of [0, 1]: values and derivatives at x.
void equispaced_basis(int g, double x, double* val, double* der) {
  const long double xl = x;
  for (int i = 0; i <= g; ++i) {
    long double v = 1.0L, d = 0.0L;
    for (int m = 0; m <= g; ++m) {
      if (m == i) continue;
      const long double den = static_cast<long double>(i - m) / g;
      const long double f = (xl - static_cast<long double>(m) / g) / den;
      d = d * f + v / den;
      v *= f;
    }
    val[i] = static_cast<double>(v);
    if (der) der[i] = static_cast<double>(d);
  }
}

// One thread per (cell, Gauss point): J0 = dX/dxi of the cell's degree-g map, K = J0^-1 and
// w det J0 into the block-interleaved planes [block][kGeoWords][EB n^3] (FP64 and FP32).
struct GeoTables {
  int n, g, eb;
  double L[8 * (kMaxGeomDegree + 1)];   // L[q (g+1) + i] = l_i(x_q) (equispaced basis, Gauss points)
  double dL[8 * (kMaxGeomDegree + 1)];
  double w[8];                          // Gauss weights
};

__global__ void k_stored_geometry(const double* __restrict__ X, int64_t n_cells, GeoTables T,
                                  double* __restrict__ geo64, float* __restrict__ geo32, int* flag) {
  const int n = T.n, m = T.g + 1;
  const int Q = n * n * n;
  const int64_t total = n_cells * Q;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t e = idx / Q;
    const int q = static_cast<int>(idx - e * Q);
    const int qx = q % n, qy = (q / n) % n, qz = q / (n * n);
    const double* Xe = X + e * (m * m * m) * 3;
    double J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < m; ++k)
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
          const double vx = T.L[qx * m + i], vy = T.L[qy * m + j], vz = T.L[qz * m + k];
          const double gx = T.dL[qx * m + i] * vy * vz, gy = vx * T.dL[qy * m + j] * vz,
                       gz = vx * vy * T.dL[qz * m + k];
          const double* P = Xe + 3 * (i + m * (j + m * k));
          for (int c = 0; c < 3; ++c) {
            J[3 * c + 0] += P[c] * gx;
            J[3 * c + 1] += P[c] * gy;
            J[3 * c + 2] += P[c] * gz;
          }
        }
    double A[9];
    A[0] = J[4] * J[8] - J[5] * J[7];
    A[1] = J[2] * J[7] - J[1] * J[8];
    A[2] = J[1] * J[5] - J[2] * J[4];
    A[3] = J[5] * J[6] - J[3] * J[8];
    A[4] = J[0] * J[8] - J[2] * J[6];
    A[5] = J[2] * J[3] - J[0] * J[5];
    A[6] = J[3] * J[7] - J[4] * J[6];
    A[7] = J[1] * J[6] - J[0] * J[7];
    A[8] = J[0] * J[4] - J[1] * J[3];
    const double det = J[0] * A[0] + J[1] * A[3] + J[2] * A[6];
    if (!(det > 0.0) || !isfinite(det)) atomicOr(flag, 1);
    double out[kGeoWords];
    for (int i = 0; i < 9; ++i) out[i] = A[i] / det;
    out[9] = T.w[qx] * T.w[qy] * T.w[qz] * det;
    const int64_t blk = e / T.eb;
    const int64_t le = e - blk * T.eb;
    const int64_t ebq = static_cast<int64_t>(T.eb) * Q;
    const int64_t base = blk * kGeoWords * ebq + le * Q + q;
    for (int w = 0; w < kGeoWords; ++w) {
      geo64[base + w * ebq] = out[w];
      geo32[base + w * ebq] = static_cast<float>(out[w]);
    }
  }
}

// ---------------------------------------------------------------- node numbering of general meshes
// Identity of a node shared between cells, from the global vertex ids of the entity it lies on:
// kind 0 vertex (a), 1 edge (ends a < b, index u from a), 2 face (corner a of smallest id, the
// corner b next to it with the smaller id, the corner c next to it on the other side, (u, v)
// in the frame a -> b, a -> c); interior nodes are never shared and are not looked up.
struct NodeKey {
  int kind;
  int64_t a, b, c;
  int u, v;
  bool operator==(const NodeKey& o) const {
    return kind == o.kind && a == o.a && b == o.b && c == o.c && u == o.u && v == o.v;
  }
};

struct NodeKeyHash {
  size_t operator()(const NodeKey& k) const {
    uint64_t h = static_cast<uint64_t>(k.kind) * 0x9e3779b97f4a7c15ull;
    const uint64_t parts[5] = {static_cast<uint64_t>(k.a), static_cast<uint64_t>(k.b), static_cast<uint64_t>(k.c),
                               static_cast<uint64_t>(k.u), static_cast<uint64_t>(k.v)};
    for (uint64_t x : parts) {
      h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
      h *= 0xbf58476d1ce4e5b9ull;
    }
    return static_cast<size_t>(h ^ (h >> 31));
  }
};

// corner id of cell-local lattice corner (a, b, c) in {0, 1}^3
inline int64_t corner(const int64_t* cv, int a, int b, int c) { return cv[a + 2 * b + 4 * c]; }

// key of the node at local index (i, j, k) of a cell of degree p with corner ids cv; false for an
// interior node
bool node_key(const int64_t* cv, int p, int i, int j, int k, NodeKey& key) {
  const int l[3] = {i, j, k};
  int nb = 0, free_dir[3], nf = 0;
  for (int d = 0; d < 3; ++d) {
    if (l[d] == 0 || l[d] == p)
      ++nb;
    else
      free_dir[nf++] = d;
  }
  if (nb == 0) return false;
  auto at = [&](const int* pos) {  // corner id at corner coordinates pos[d] in {0, 1}
    return corner(cv, pos[0], pos[1], pos[2]);
  };
  int base[3];
  for (int d = 0; d < 3; ++d) base[d] = l[d] == p ? 1 : 0;
  if (nb == 3) {
    key = NodeKey{0, at(base), 0, 0, 0, 0};
    return true;
  }
  if (nb == 2) {
    const int d = free_dir[0];
    int p0[3] = {base[0], base[1], base[2]}, p1[3] = {base[0], base[1], base[2]};
    p0[d] = 0;
    p1[d] = 1;
    int64_t va = at(p0), vb = at(p1);
    int u = l[d];
    if (va > vb) {
      std::swap(va, vb);
      u = p - u;
    }
    key = NodeKey{1, va, vb, 0, u, 0};
    return true;
  }
  // face node: in-face directions d1 < d2, corners at (s, t) in {0, 1}^2 of the face
  const int d1 = free_dir[0], d2 = free_dir[1];
  int64_t id[2][2];
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t) {
      int pos[3] = {base[0], base[1], base[2]};
      pos[d1] = s;
      pos[d2] = t;
      id[s][t] = at(pos);
    }
  // the eight symmetries of the face: (s, t) -> new position; choose the one that puts the
  // smallest id at the origin and its smaller neighbour on the first axis
  int best = -1;
  NodeKey bk{};
  for (int sym = 0; sym < 8; ++sym) {
    auto map = [&](int s, int t, int pp, int& s2, int& t2) {
      int a = s, b = t;
      if (sym & 4) std::swap(a, b);
      if (sym & 1) a = pp - a;
      if (sym & 2) b = pp - b;
      s2 = a;
      t2 = b;
    };
    int64_t nid[2][2];
    for (int s = 0; s < 2; ++s)
      for (int t = 0; t < 2; ++t) {
        int s2, t2;
        map(s, t, 1, s2, t2);
        nid[s2][t2] = id[s][t];
      }
    int u, v;
    map(l[d1], l[d2], p, u, v);
    const NodeKey cand{2, nid[0][0], nid[1][0], nid[0][1], u, v};
    if (best < 0 || cand.a < bk.a || (cand.a == bk.a && cand.b < bk.b)) {
      best = sym;
      bk = cand;
    }
  }
  key = bk;
  return true;
}

}  // namespace

int64_t host_node(const hx_ctx_s* c, int64_t e, int i, int j, int k) {
  const int n = c->p + 1;
  if (c->topo == kTopoMap) return c->cell_nodes[static_cast<size_t>(e) * n * n * n + i + n * (j + n * k)];
  const Lattice& L = c->L;
  const int64_t ex = e % L.nx, ey = (e / L.nx) % L.ny, ez = e / (static_cast<int64_t>(L.nx) * L.ny);
  int64_t I = ex * c->p + i, J = ey * c->p + j, K = ez * c->p + k;
  I = I >= L.Nx ? I - L.Nx : I;
  J = J >= L.Ny ? J - L.Ny : J;
  K = K >= L.Nz ? K - L.Nz : K;
  return I + static_cast<int64_t>(L.Nx) * (J + static_cast<int64_t>(L.Ny) * K);
}

void host_map(const hx_ctx_s* c, int64_t e, const double* xi, double* X, double* dX) {
  const bool tri = c->topo == kTopoLattice;
  const int g = tri ? 1 : c->geom_degree;
  const int m = g + 1;
  double val[3][kMaxGeomDegree + 1], der[3][kMaxGeomDegree + 1];
  for (int d = 0; d < 3; ++d) equispaced_basis(g, xi[d], val[d], der[d]);
  const double* P = nullptr;
  double corners[8 * 3];
  if (tri) {
    // the 8 vertices of a lattice cell, corner a + 2b + 4c
    const Lattice& L = c->L;
    const int64_t ex = e % L.nx, ey = (e / L.nx) % L.ny, ez = e / (static_cast<int64_t>(L.nx) * L.ny);
    for (int v = 0; v < 8; ++v) {
      int64_t vx = ex + (v & 1), vy = ey + ((v >> 1) & 1), vz = ez + (v >> 2);
      vx = vx >= L.Vx ? vx - L.Vx : vx;
      vy = vy >= L.Vy ? vy - L.Vy : vy;
      vz = vz >= L.Vz ? vz - L.Vz : vz;
      const double* src = &c->vert_host[3 * (vx + static_cast<int64_t>(L.Vx) * (vy + static_cast<int64_t>(L.Vy) * vz))];
      for (int k = 0; k < 3; ++k) corners[3 * v + k] = src[k];
    }
    P = corners;
  } else {
    P = c->geom_host.data() + static_cast<size_t>(e) * m * m * m * 3;
  }
  for (int k = 0; k < 3; ++k) X[k] = 0.0;
  if (dX)
    for (int k = 0; k < 9; ++k) dX[k] = 0.0;
  for (int kk = 0; kk < m; ++kk)
    for (int jj = 0; jj < m; ++jj)
      for (int ii = 0; ii < m; ++ii) {
        const double* Pa = P + 3 * (ii + m * (jj + m * kk));
        const double w = val[0][ii] * val[1][jj] * val[2][kk];
        for (int k = 0; k < 3; ++k) X[k] += w * Pa[k];
        if (dX) {
          const double g0 = der[0][ii] * val[1][jj] * val[2][kk];
          const double g1 = val[0][ii] * der[1][jj] * val[2][kk];
          const double g2 = val[0][ii] * val[1][jj] * der[2][kk];
          for (int k = 0; k < 3; ++k) {
            dX[3 * k + 0] += g0 * Pa[k];
            dX[3 * k + 1] += g1 * Pa[k];
            dX[3 * k + 2] += g2 * Pa[k];
          }
        }
      }
}

hx_status build_stored_geometry(hx_ctx_s* c) {
  const int p = c->p, n = p + 1, g = c->geom_degree;
  const int64_t cells = c->L.n_cells;
  const int64_t Q = static_cast<int64_t>(n) * n * n;
  const int64_t eb = cells_per_block(p);
  const int64_t nblk = (cells + eb - 1) / eb;
  const size_t planes = static_cast<size_t>(nblk) * kGeoWords * eb * Q;
  GeoTables T{};
  T.n = n;
  T.g = g;
  T.eb = static_cast<int>(eb);
  for (int q = 0; q < n; ++q) {
    equispaced_basis(g, c->base.x[q], T.L + q * (g + 1), T.dL + q * (g + 1));
    T.w[q] = c->base.w[q];
  }
  double* X = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&c->geo64, planes * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->geo32, planes * sizeof(float))) != hipSuccess ||
      (e = hipMemset(c->geo64, 0, planes * sizeof(double))) != hipSuccess ||
      (e = hipMemset(c->geo32, 0, planes * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&X, c->geom_host.size() * sizeof(double))) != hipSuccess ||
      (e = hipMemcpy(X, c->geom_host.data(), c->geom_host.size() * sizeof(double), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemset(c->flag, 0, sizeof(int))) != hipSuccess) {
    if (X) (void)hipFree(X);
    c->err = std::string("hx_setup: stored geometry: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? HX_E_NOMEM : HX_E_HIP;
  }
  const int64_t total = cells * Q;
  const unsigned grid = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536)));
  k_stored_geometry<<<grid, 256>>>(X, cells, T, c->geo64, c->geo32, c->flag);
  int flag = 0;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost);
  (void)hipFree(X);
  if (e != hipSuccess) {
    c->err = std::string("hx_setup: stored geometry: ") + hipGetErrorString(e);
    return HX_E_HIP;
  }
  if (flag) {
    c->err = "hx_setup: det J0 <= 0 (or not finite) at a Gauss point of some cell";
    return HX_E_INVERTED;
  }
  return hipMemset(c->flag, 0, sizeof(int)) == hipSuccess ? HX_OK : HX_E_HIP;
}

}  // namespace hx

using namespace hx;

extern "C" hx_status hx_setup(const hx_mesh* mesh, int32_t p, const hx_material* mat, const hx_options* opt,
                              hx_ctx* out) {
  if (!out) return setup_fail(HX_E_ARG, "hx_setup: out is NULL");
  *out = nullptr;
  if (!mesh || !mat || !mesh->cells) return setup_fail(HX_E_ARG, "hx_setup: NULL mesh, cells or material");
  if (p < 1 || p > kMaxDegree) return setup_fail(HX_E_UNSUPPORTED, "hx_setup: degree must be in [1, 6]");
  if (mat->law != HX_LAW_CNH && mat->law != HX_LAW_INH && mat->law != HX_LAW_FIBER)
    return setup_fail(HX_E_ARG, "hx_setup: unknown law");
  if (!check_options(opt, "hx_setup")) return HX_E_ARG;
  const int64_t nv = mesh->n_vertices, cells = mesh->n_cells;
  if (cells < 1 || nv < 8) return setup_fail(HX_E_ARG, "hx_setup: a mesh needs at least one cell and 8 vertices");
  if (!mesh->vertices) return setup_fail(HX_E_ARG, "hx_setup: NULL vertices");
  const int g = mesh->geom_degree;
  if (g < 1 || g > kMaxGeomDegree) return setup_fail(HX_E_ARG, "hx_setup: geom_degree out of [1, 8]");
  if (g > 1 && !mesh->geom_nodes) return setup_fail(HX_E_ARG, "hx_setup: geom_degree > 1 needs geom_nodes");
  const int n = p + 1;
  const int64_t Q = static_cast<int64_t>(n) * n * n;
  const int64_t eb = cells_per_block(p);
  if ((cells + eb) * Q > (int64_t(1) << 31) - 1)
    return setup_fail(HX_E_ARG, "hx_setup: mesh too large (cells * (p+1)^3 must fit in int32)");
  const uint32_t bid_mask = opt ? opt->dirichlet_bid_mask : 0u;
  if (bid_mask & 1u) return setup_fail(HX_E_ARG, "hx_setup: boundary id 0 means no boundary and cannot be constrained");
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(mesh->vertices[i])) return setup_fail(HX_E_ARG, "hx_setup: non-finite vertex coordinate");
  for (int64_t e = 0; e < cells; ++e) {
    const int64_t* cv = mesh->cells + 8 * e;
    for (int a = 0; a < 8; ++a) {
      if (cv[a] < 0 || cv[a] >= nv) return setup_fail(HX_E_ARG, "hx_setup: vertex id out of range in cell " + std::to_string(e));
      for (int b = 0; b < a; ++b)
        if (cv[a] == cv[b]) return setup_fail(HX_E_ARG, "hx_setup: cell " + std::to_string(e) + " repeats a vertex");
    }
  }

  hx_ctx_s* c = new (std::nothrow) hx_ctx_s();
  if (!c) return setup_fail(HX_E_NOMEM, "hx_setup: host allocation failed");
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return setup_fail(HX_E_HIP, "hx_setup: no HIP device");
  }
  c->p = p;
  c->topo = kTopoMap;
  c->geom_degree = g;

  // first-touch numbering: cells in order, local nodes x fastest; shared nodes by their keys
  try {
    c->cell_nodes.assign(static_cast<size_t>(cells * Q), 0);
    std::unordered_map<NodeKey, int32_t, NodeKeyHash> ids;
    ids.reserve(static_cast<size_t>(cells) * (Q - (p > 1 ? (p - 1) * (p - 1) * (p - 1) : 0)));
    int64_t next = 0;
    for (int64_t e = 0; e < cells; ++e) {
      const int64_t* cv = mesh->cells + 8 * e;
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            NodeKey key;
            int64_t id;
            if (!node_key(cv, p, i, j, k, key)) {
              id = next++;
            } else {
              auto it = ids.find(key);
              if (it == ids.end()) {
                id = next++;
                if (id > INT32_MAX) throw std::bad_alloc();
                ids.emplace(key, static_cast<int32_t>(id));
              } else {
                id = it->second;
              }
            }
            if (id > INT32_MAX) throw std::bad_alloc();
            c->cell_nodes[static_cast<size_t>(e * Q + i + n * (j + n * k))] = static_cast<int32_t>(id);
          }
    }
    c->L.n_nodes = next;
    // constraints: every node on a face whose boundary id is in the mask
    c->cons_host.assign(static_cast<size_t>(next), 0);
    c->face_bid.assign(static_cast<size_t>(6 * cells), 0);
    if (mesh->face_bid) std::memcpy(c->face_bid.data(), mesh->face_bid, static_cast<size_t>(6 * cells));
    for (int64_t e = 0; e < cells; ++e)
      for (int f = 0; f < 6; ++f) {
        const uint8_t b = c->face_bid[static_cast<size_t>(6 * e + f)];
        if (b == 0 || b > 31 || !((bid_mask >> b) & 1u)) continue;
        const int d = f / 2, side = f % 2;
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              const int l[3] = {i, j, k};
              if (l[d] != (side ? p : 0)) continue;
              c->cons_host[c->cell_nodes[static_cast<size_t>(e * Q + i + n * (j + n * k))]] = 1;
            }
      }
    // geometry points of every cell: given, or the 8 vertices (degree 1, corner a + 2b + 4c is the
    // equispaced point (a, b, c))
    const size_t m3 = static_cast<size_t>(g + 1) * (g + 1) * (g + 1);
    if (mesh->geom_nodes) {
      c->geom_host.assign(mesh->geom_nodes, mesh->geom_nodes + 3 * m3 * cells);
    } else {
      c->geom_host.resize(static_cast<size_t>(24 * cells));
      for (int64_t e = 0; e < cells; ++e)
        for (int a = 0; a < 8; ++a)
          for (int k = 0; k < 3; ++k) c->geom_host[24 * e + 3 * a + k] = mesh->vertices[3 * mesh->cells[8 * e + a] + k];
    }
  } catch (const std::bad_alloc&) {
    delete c;
    return setup_fail(HX_E_NOMEM, "hx_setup: host memory for the node numbering (or more than 2^31 nodes)");
  }
  for (double v : c->geom_host)
    if (!std::isfinite(v)) {
      delete c;
      return setup_fail(HX_E_ARG, "hx_setup: non-finite geometry point");
    }
  Lattice& L = c->L;
  // the lattice fields are unused by general meshes; set to a harmless 1D arrangement
  L.nx = static_cast<int32_t>(cells);
  L.ny = L.nz = 1;
  L.Vx = L.Vy = L.Vz = 1;
  L.Nx = static_cast<int32_t>(std::min<int64_t>(L.n_nodes, INT32_MAX));
  L.Ny = L.Nz = 1;
  L.p = p;
  L.dir_faces = 0;
  L.n_cells = static_cast<int32_t>(cells);

  // gather map in the element kernel's thread order, and each node's slots in increasing order
  const int64_t nblk = (cells + eb - 1) / eb;
  const int64_t slots = nblk * eb * Q;
  std::vector<int32_t> map(static_cast<size_t>(slots), 0);
  std::vector<int32_t> nptr(static_cast<size_t>(L.n_nodes) + 1, 0);
  for (int64_t b = 0; b < nblk; ++b)
    for (int t = 0; t < eb * Q; ++t) {
      int le, q;
      slot_of_thread(n, static_cast<int>(eb), t, le, q);
      const int64_t e = b * eb + le;
      if (e >= cells) continue;
      const int32_t node = c->cell_nodes[static_cast<size_t>(e * Q + q)];
      const bool cons = c->cons_host[node] != 0;
      map[static_cast<size_t>(b * eb * Q + t)] = cons ? ~node : node;
      if (!cons) ++nptr[static_cast<size_t>(node) + 1];
    }
  for (int64_t i = 0; i < L.n_nodes; ++i) nptr[static_cast<size_t>(i) + 1] += nptr[static_cast<size_t>(i)];
  std::vector<int32_t> nslot(static_cast<size_t>(nptr.back()) + 1, 0);
  {
    std::vector<int32_t> fill(nptr.begin(), nptr.end() - 1);
    for (int64_t s = 0; s < slots; ++s) {
      const int64_t b = s / (eb * Q);
      int le, q;
      slot_of_thread(n, static_cast<int>(eb), static_cast<int>(s - b * eb * Q), le, q);
      const int64_t e = b * eb + le;
      if (e >= cells) continue;
      const int32_t v = map[static_cast<size_t>(s)];
      if (v < 0) continue;
      nslot[static_cast<size_t>(fill[v]++)] = static_cast<int32_t>(s);
    }
  }
  hipError_t e;
  if ((e = hipMalloc(&c->map, map.size() * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc(&c->nptr, nptr.size() * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc(&c->nslot, nslot.size() * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc(&c->cmask, c->cons_host.size())) != hipSuccess ||
      (e = hipMemcpy(c->map, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->nptr, nptr.data(), nptr.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->nslot, nslot.data(), nslot.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->cmask, c->cons_host.data(), c->cons_host.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    hx_destroy(c);
    return setup_fail(e == hipErrorOutOfMemory ? HX_E_NOMEM : HX_E_HIP, std::string("hx_setup: mesh arrays: ") + hipGetErrorString(e));
  }
  return finish_setup(c, mat, opt, mesh->frames, out);
}

// ---------------------------------------------------------------- pressure loads
// f_(c,a) = -pressure * int phi_a N_c dA over the listed (cell, local face) pairs, (p+1)^2 Gauss
// points per face of the cell's map; the outward area element of local face f = (d, side) is
// sign (dX/dxi_a x dX/dxi_b), (a, b) = (d + 1, d + 2) mod 3, sign +1 on the side xi_d = 1.
namespace {

void face_loads(const hx_ctx_s* ctx, const std::vector<std::array<int64_t, 2>>& faces, double pressure, double* f) {
  const int n = ctx->p + 1;
  const int64_t nn = ctx->L.n_nodes;
  const double* xq = ctx->base.x;
  const double* wq = ctx->base.w;
  std::vector<double> la(n * n);  // la[q*n + i] = l_i(x_q) on the GLL nodes
  for (int qq = 0; qq < n; ++qq)
    for (int i = 0; i < n; ++i) {
      double v = 1.0;
      for (int m = 0; m < n; ++m)
        if (m != i) v *= (xq[qq] - ctx->gll[m]) / (ctx->gll[i] - ctx->gll[m]);
      la[qq * n + i] = v;
    }
  for (const auto& cf : faces) {
    const int64_t e = cf[0];
    const int face = static_cast<int>(cf[1]);
    const int d = face / 2, side = face % 2;
    const int da = (d + 1) % 3, db = (d + 2) % 3;
    for (int q2 = 0; q2 < n; ++q2)
      for (int q1 = 0; q1 < n; ++q1) {
        double xi[3];
        xi[d] = side ? 1.0 : 0.0;
        xi[da] = xq[q1];
        xi[db] = xq[q2];
        double X[3], dX[9];
        host_map(ctx, e, xi, X, dX);
        const double ta[3] = {dX[da], dX[3 + da], dX[6 + da]};
        const double tb[3] = {dX[db], dX[3 + db], dX[6 + db]};
        const double nda[3] = {ta[1] * tb[2] - ta[2] * tb[1], ta[2] * tb[0] - ta[0] * tb[2], ta[0] * tb[1] - ta[1] * tb[0]};
        const double sgn = side ? 1.0 : -1.0;
        const double w = wq[q1] * wq[q2];
        for (int j2 = 0; j2 < n; ++j2)
          for (int j1 = 0; j1 < n; ++j1) {
            int loc[3];
            loc[d] = side ? n - 1 : 0;
            loc[da] = j1;
            loc[db] = j2;
            const int64_t node = host_node(ctx, e, loc[0], loc[1], loc[2]);
            const double phi = la[q1 * n + j1] * la[q2 * n + j2];
            for (int k = 0; k < 3; ++k) f[k * nn + node] += -pressure * sgn * nda[k] * w * phi;
          }
      }
  }
}

}  // namespace

// Dead-load pressure (Section 2, Neumann term of the residual): on lattice face `face` (0..5) of a
// lattice context, or on the cell faces with boundary id `face` (1..255) of a general mesh.
extern "C" hx_status hx_surface_load(hx_ctx ctx, int32_t face, double pressure, double* f) {
  if (!ctx || !f) return HX_E_ARG;
  const int64_t nn = ctx->L.n_nodes;
  std::vector<std::array<int64_t, 2>> faces;
  if (ctx->topo == kTopoMap) {
    if (face < 1 || face > 255) return set_error(ctx, HX_E_ARG, "hx_surface_load: boundary id out of [1, 255]");
    for (int64_t e = 0; e < ctx->L.n_cells; ++e)
      for (int lf = 0; lf < 6; ++lf)
        if (ctx->face_bid[static_cast<size_t>(6 * e + lf)] == face) faces.push_back({e, lf});
  } else {
    if (face < 0 || face > 5) return set_error(ctx, HX_E_ARG, "hx_surface_load: face out of [0, 5]");
    const Lattice& L = ctx->L;
    const int d = face / 2, side = face % 2;
    const int per = (L.Nx == L.nx * L.p ? 1 : 0) | (L.Ny == L.ny * L.p ? 2 : 0) | (L.Nz == L.nz * L.p ? 4 : 0);
    if (per & (1 << d)) return set_error(ctx, HX_E_ARG, "hx_surface_load: face of a periodic direction");
    const int nc[3] = {L.nx, L.ny, L.nz};
    const int da = (d + 1) % 3, db = (d + 2) % 3;
    const int cd = side ? nc[d] - 1 : 0;
    for (int c2 = 0; c2 < nc[db]; ++c2)
      for (int c1 = 0; c1 < nc[da]; ++c1) {
        int cell[3];
        cell[d] = cd;
        cell[da] = c1;
        cell[db] = c2;
        faces.push_back({cell[0] + static_cast<int64_t>(L.nx) * (cell[1] + static_cast<int64_t>(L.ny) * cell[2]), face});
      }
  }
  std::memset(f, 0, 3 * nn * sizeof(double));
  face_loads(ctx, faces, pressure, f);
  return HX_OK;
}
