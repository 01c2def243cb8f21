// Icosphere surface description (nodal discretisation of the scatterer
// surfaces; Sec. IV A meshes the sphere with triangular elements and collocates
// at the nodes).  Host code, compiled without floating-point contraction so
// that every value is reproducible bit for bit: each expression is evaluated
// in the written order with correctly rounded IEEE operations.
#include <cmath>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "../../include/bem.h"

namespace {

struct V3 {
  double x, y, z;
};

V3 unit(V3 v) {
  double s = std::sqrt((v.x * v.x + v.y * v.y) + v.z * v.z);
  return {v.x / s, v.y / s, v.z / s};
}

const double kPhi = (1.0 + std::sqrt(5.0)) / 2.0;

void base_icosahedron(std::vector<V3>& v, std::vector<int32_t>& f) {
  const double p = kPhi;
  const V3 raw[12] = {{-1, p, 0}, {1, p, 0},  {-1, -p, 0}, {1, -p, 0}, {0, -1, p},  {0, 1, p},
                      {0, -1, -p}, {0, 1, -p}, {p, 0, -1},  {p, 0, 1},  {-p, 0, -1}, {-p, 0, 1}};
  static const int32_t tri[60] = {0, 11, 5, 0, 5,  1,  0, 1, 7, 0, 7,  10, 0, 10, 11,
                                  1, 5,  9, 5, 11, 4,  11, 10, 2, 10, 7, 6, 7, 1,  8,
                                  3, 9,  4, 3, 4,  2,  3, 2, 6, 3, 6,  8,  3, 8,  9,
                                  4, 9,  5, 2, 4,  11, 6, 2, 10, 8, 6, 7, 9, 8,  1};
  v.clear();
  for (int i = 0; i < 12; ++i) v.push_back(unit(raw[i]));
  f.assign(tri, tri + 60);
}

void subdivide(std::vector<V3>& v, std::vector<int32_t>& f) {
  std::unordered_map<uint64_t, int32_t> cache;
  cache.reserve(f.size());
  std::vector<int32_t> nf;
  nf.reserve(f.size() * 4);
  auto mid = [&](int32_t a, int32_t b) -> int32_t {
    uint64_t key = a < b ? ((uint64_t)a << 32) | (uint32_t)b : ((uint64_t)b << 32) | (uint32_t)a;
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    V3 pa = v[a], pb = v[b];
    V3 m = {(pa.x + pb.x) * 0.5, (pa.y + pb.y) * 0.5, (pa.z + pb.z) * 0.5};
    v.push_back(unit(m));
    int32_t idx = (int32_t)v.size() - 1;
    cache.emplace(key, idx);
    return idx;
  };
  for (size_t t = 0; t < f.size(); t += 3) {
    int32_t a = f[t], b = f[t + 1], c = f[t + 2];
    int32_t ab = mid(a, b);
    int32_t bc = mid(b, c);
    int32_t ca = mid(c, a);
    const int32_t kids[12] = {a, ab, ca, b, bc, ab, c, ca, bc, ab, bc, ca};
    nf.insert(nf.end(), kids, kids + 12);
  }
  f.swap(nf);
}

double spheroid_area(double radius, double aspect) {
  if (aspect == 1.0) return 4.0 * M_PI * radius * radius;
  double a = radius;
  double c = radius * aspect;
  double e = std::sqrt(1.0 - (a * a) / (c * c));
  return 2.0 * M_PI * a * a * (1.0 + (c / (a * e)) * std::asin(e));
}

}  // namespace

extern "C" bem_status bem_mesh_counts(int32_t level, int32_t* nv, int32_t* nf) {
  if (level < 0 || level > 7 || !nv || !nf) return BEM_EINVAL;
  int64_t p = 1;
  for (int i = 0; i < level; ++i) p *= 4;
  *nv = (int32_t)(10 * p + 2);
  *nf = (int32_t)(20 * p);
  return BEM_OK;
}

extern "C" bem_status bem_mesh_icosphere(int32_t level, double radius, double aspect,
                                         const double center[3], int32_t rescale_area, double* x,
                                         double* nrm, double* w, int32_t* faces) {
  if (level < 0 || level > 7 || !(radius > 0.0) || !(aspect >= 1.0) || !std::isfinite(radius) ||
      !std::isfinite(aspect) || !center || !x || !nrm || !w)
    return BEM_EINVAL;
  std::vector<V3> u;
  std::vector<int32_t> f;
  base_icosahedron(u, f);
  for (int l = 0; l < level; ++l) subdivide(u, f);
  const size_t V = u.size();
  const double cx = center[0], cy = center[1], cz = center[2];
  const double sx = radius;
  const double sz = radius * aspect;
  for (size_t i = 0; i < V; ++i) {
    x[3 * i + 0] = cx + sx * u[i].x;
    x[3 * i + 1] = cy + sx * u[i].y;
    x[3 * i + 2] = cz + sz * u[i].z;
    V3 g = {u[i].x / sx, u[i].y / sx, u[i].z / sz};
    V3 n = unit(g);
    nrm[3 * i + 0] = n.x;
    nrm[3 * i + 1] = n.y;
    nrm[3 * i + 2] = n.z;
    w[i] = 0.0;
  }
  double total = 0.0;
  for (size_t t = 0; t < f.size(); t += 3) {
    const double* pa = x + 3 * f[t];
    const double* pb = x + 3 * f[t + 1];
    const double* pc = x + 3 * f[t + 2];
    double e1x = pb[0] - pa[0], e1y = pb[1] - pa[1], e1z = pb[2] - pa[2];
    double e2x = pc[0] - pa[0], e2y = pc[1] - pa[1], e2z = pc[2] - pa[2];
    double c0 = e1y * e2z - e1z * e2y;
    double c1 = e1z * e2x - e1x * e2z;
    double c2 = e1x * e2y - e1y * e2x;
    double area = 0.5 * std::sqrt((c0 * c0 + c1 * c1) + c2 * c2);
    total = total + area;
    double third = area / 3.0;
    w[f[t]] = w[f[t]] + third;
    w[f[t + 1]] = w[f[t + 1]] + third;
    w[f[t + 2]] = w[f[t + 2]] + third;
  }
  if (rescale_area) {
    double factor = spheroid_area(radius, aspect) / total;
    for (size_t i = 0; i < V; ++i) w[i] = w[i] * factor;
  }
  if (faces)
    for (size_t t = 0; t < f.size(); ++t) faces[t] = f[t];
  return BEM_OK;
}

// The axisymmetric bowl of Sec. IV C (Eq. dish): the closed meridian curve
// xi = a sin(theta), eta = a (0.2 cos(theta) - 0.6 sin^2(theta)) rotated about
// the eta axis, meshed by poles and rings of constant theta.
extern "C" bem_status bem_mesh_bowl_counts(int32_t n_theta, int32_t n_phi, int32_t* n_vertices,
                                           int32_t* n_faces) {
  if (n_theta < 2 || n_phi < 3 || n_theta > 4096 || n_phi > 8192 || !n_vertices || !n_faces)
    return BEM_EINVAL;
  *n_vertices = 2 + (n_theta - 1) * n_phi;
  *n_faces = 2 * n_phi * (n_theta - 1);
  return BEM_OK;
}

extern "C" bem_status bem_mesh_bowl(int32_t n_theta, int32_t n_phi, double radius, double tilt,
                                    const double center[3], double* x, double* nrm, double* w,
                                    int32_t* faces) {
  int32_t V = 0, F = 0;
  if (bem_mesh_bowl_counts(n_theta, n_phi, &V, &F) != BEM_OK || !(radius > 0.0) ||
      !std::isfinite(radius) || !std::isfinite(tilt) || !center || !x || !nrm || !w)
    return BEM_EINVAL;
  const double ct = std::cos(tilt), st = std::sin(tilt);
  const double cx = center[0], cy = center[1], cz = center[2];
  auto place = [&](int k, double px, double py, double pz, double qx, double qy, double qz) {
    x[3 * k + 0] = cx + px;
    x[3 * k + 1] = cy + (py * ct - pz * st);
    x[3 * k + 2] = cz + (py * st + pz * ct);
    nrm[3 * k + 0] = qx;
    nrm[3 * k + 1] = qy * ct - qz * st;
    nrm[3 * k + 2] = qy * st + qz * ct;
  };
  place(0, 0.0, 0.0, radius * (0.2 * std::cos(0.0)), 0.0, 0.0, 1.0);
  int k = 1;
  for (int i = 1; i < n_theta; ++i) {
    const double th = (M_PI * i) / n_theta;
    const double s = std::sin(th), c = std::cos(th);
    const double xi = radius * s;
    const double eta = radius * (0.2 * c - 0.6 * (s * s));
    // outward normal of the meridian curve: (-eta', xi') / |(xi', eta')|
    const double dxi = c;
    const double deta = -0.2 * s - 1.2 * (s * c);
    const double m = std::sqrt(dxi * dxi + deta * deta);
    const double nxi = -deta / m, neta = dxi / m;
    for (int j = 0; j < n_phi; ++j) {
      const double ph = (2.0 * M_PI * j) / n_phi;
      const double cp = std::cos(ph), sp = std::sin(ph);
      place(k++, xi * cp, xi * sp, eta, nxi * cp, nxi * sp, neta);
    }
  }
  place(V - 1, 0.0, 0.0, radius * (0.2 * std::cos(M_PI)), 0.0, 0.0, -1.0);
  std::vector<int32_t> f;
  f.reserve(3 * (size_t)F);
  auto tri = [&](int a, int b, int c) { f.push_back(a); f.push_back(b); f.push_back(c); };
  for (int j = 0; j < n_phi; ++j) tri(0, 1 + j, 1 + (j + 1) % n_phi);
  for (int i = 1; i < n_theta - 1; ++i) {
    const int r0 = 1 + (i - 1) * n_phi, r1 = r0 + n_phi;
    for (int j = 0; j < n_phi; ++j) {
      const int j1 = (j + 1) % n_phi;
      tri(r0 + j, r1 + j, r1 + j1);
      tri(r0 + j, r1 + j1, r0 + j1);
    }
  }
  const int rl = 1 + (n_theta - 2) * n_phi;
  for (int j = 0; j < n_phi; ++j) tri(V - 1, rl + (j + 1) % n_phi, rl + j);
  for (int v = 0; v < V; ++v) w[v] = 0.0;
  for (size_t t = 0; t < f.size(); t += 3) {
    const double* pa = x + 3 * f[t];
    const double* pb = x + 3 * f[t + 1];
    const double* pc = x + 3 * f[t + 2];
    const double e1x = pb[0] - pa[0], e1y = pb[1] - pa[1], e1z = pb[2] - pa[2];
    const double e2x = pc[0] - pa[0], e2y = pc[1] - pa[1], e2z = pc[2] - pa[2];
    const double c0 = e1y * e2z - e1z * e2y;
    const double c1 = e1z * e2x - e1x * e2z;
    const double c2 = e1x * e2y - e1y * e2x;
    const double third = (0.5 * std::sqrt((c0 * c0 + c1 * c1) + c2 * c2)) / 3.0;
    w[f[t]] = w[f[t]] + third;
    w[f[t + 1]] = w[f[t + 1]] + third;
    w[f[t + 2]] = w[f[t + 2]] + third;
  }
  if (faces)
    for (size_t t = 0; t < f.size(); ++t) faces[t] = f[t];
  return BEM_OK;
}

// Six-node quadratic elements on a frequency-nu geodesic sphere (Sec. III:
// quadratic interpolation within each element; Sec. IV A: 500 elements and
// 1002 nodes, i.e. nu = 5).  Each icosahedron face is cut into nu^2 triangles
// on its barycentric grid; a grid point with integer weights (c_A, c_B, c_C)
// is shared between faces through its nonzero (vertex, weight) pairs and
// placed at normalise(sum c_v V_v), summed in increasing vertex index.  The
// elements' edge midpoints (chord midpoints projected onto the sphere) follow
// the vertices, in the order met walking each element's edges (v0 v1),
// (v1 v2), (v2 v0).  Element nodes: (v0, v1, v2, m01, m12, m20).
namespace {

void geodesic(int nu, std::vector<V3>& pts, std::vector<int32_t>& f) {
  std::vector<V3> ico;
  std::vector<int32_t> tri;
  base_icosahedron(ico, tri);
  pts.clear();
  f.clear();
  std::unordered_map<uint64_t, int32_t> index;
  auto point = [&](int a, int b, int c, int i, int j) -> int32_t {
    // nonzero (vertex, weight) pairs in increasing vertex order
    int pv[3] = {a, b, c}, pw[3] = {nu - i - j, i, j};
    int cnt = 0, kv[3], kw[3];
    for (int s = 0; s < 3; ++s)
      if (pw[s] > 0) {
        kv[cnt] = pv[s];
        kw[cnt] = pw[s];
        ++cnt;
      }
    for (int s = 1; s < cnt; ++s)
      for (int t = s; t > 0 && (kv[t] < kv[t - 1] || (kv[t] == kv[t - 1] && kw[t] < kw[t - 1])); --t) {
        std::swap(kv[t], kv[t - 1]);
        std::swap(kw[t], kw[t - 1]);
      }
    uint64_t key = 0;
    for (int s = 0; s < 3; ++s) {
      const uint64_t slot = s < cnt ? (uint64_t)kv[s] * 4096u + (uint64_t)kw[s] : 0xFFFFu;
      key |= slot << (16 * s);
    }
    auto it = index.find(key);
    if (it != index.end()) return it->second;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int s = 0; s < cnt; ++s) {
      const double w = (double)kw[s];
      sx = sx + w * ico[kv[s]].x;
      sy = sy + w * ico[kv[s]].y;
      sz = sz + w * ico[kv[s]].z;
    }
    pts.push_back(unit({sx, sy, sz}));
    const int32_t idx = (int32_t)pts.size() - 1;
    index.emplace(key, idx);
    return idx;
  };
  std::vector<int32_t> grid((size_t)(nu + 1) * (nu + 1));
  for (int t = 0; t < 20; ++t) {
    const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    for (int i = 0; i <= nu; ++i)
      for (int j = 0; j <= nu - i; ++j) grid[(size_t)i * (nu + 1) + j] = point(a, b, c, i, j);
    auto g = [&](int i, int j) { return grid[(size_t)i * (nu + 1) + j]; };
    for (int i = 0; i < nu; ++i)
      for (int j = 0; j < nu - i; ++j) {
        const int32_t up[3] = {g(i, j), g(i + 1, j), g(i, j + 1)};
        f.insert(f.end(), up, up + 3);
        if (i + j < nu - 1) {
          const int32_t dn[3] = {g(i + 1, j), g(i + 1, j + 1), g(i, j + 1)};
          f.insert(f.end(), dn, dn + 3);
        }
      }
  }
}

}  // namespace

extern "C" bem_status bem_mesh_quadratic_counts(int32_t nu, int32_t* n_nodes, int32_t* n_elems) {
  if (nu < 1 || nu > 64 || !n_nodes || !n_elems) return BEM_EINVAL;
  *n_nodes = 40 * nu * nu + 2;
  *n_elems = 20 * nu * nu;
  return BEM_OK;
}

extern "C" bem_status bem_mesh_quadratic(int32_t nu, double radius, double aspect,
                                         const double center[3], double* x, double* nrm,
                                         int32_t* elems) {
  int32_t N = 0, F = 0;
  if (bem_mesh_quadratic_counts(nu, &N, &F) != BEM_OK || !(radius > 0.0) || !(aspect >= 1.0) ||
      !std::isfinite(radius) || !std::isfinite(aspect) || !center || !x || !nrm || !elems)
    return BEM_EINVAL;
  std::vector<V3> u;
  std::vector<int32_t> f;
  geodesic(nu, u, f);
  std::unordered_map<uint64_t, int32_t> mids;
  for (size_t t = 0; t < f.size(); t += 3) {
    const int32_t v[3] = {f[t], f[t + 1], f[t + 2]};
    int32_t m[3];
    for (int s = 0; s < 3; ++s) {
      const int32_t p = v[s], q = v[(s + 1) % 3];
      const uint64_t key = p < q ? ((uint64_t)p << 32) | (uint32_t)q : ((uint64_t)q << 32) | (uint32_t)p;
      auto it = mids.find(key);
      if (it != mids.end()) {
        m[s] = it->second;
      } else {
        const V3 pa = u[p], pb = u[q];
        u.push_back(unit({(pa.x + pb.x) * 0.5, (pa.y + pb.y) * 0.5, (pa.z + pb.z) * 0.5}));
        m[s] = (int32_t)u.size() - 1;
        mids.emplace(key, m[s]);
      }
    }
    int32_t* e = elems + 2 * t;   // element t/3, six entries
    e[0] = v[0];
    e[1] = v[1];
    e[2] = v[2];
    e[3] = m[0];
    e[4] = m[1];
    e[5] = m[2];
  }
  if ((int32_t)u.size() != N) return BEM_EINVAL;
  const double cx = center[0], cy = center[1], cz = center[2];
  const double sx = radius, sz = radius * aspect;
  for (int32_t i = 0; i < N; ++i) {
    x[3 * i + 0] = cx + sx * u[i].x;
    x[3 * i + 1] = cy + sx * u[i].y;
    x[3 * i + 2] = cz + sz * u[i].z;
    const V3 n = unit({u[i].x / sx, u[i].y / sx, u[i].z / sz});
    nrm[3 * i + 0] = n.x;
    nrm[3 * i + 1] = n.y;
    nrm[3 * i + 2] = n.z;
  }
  return BEM_OK;
}
