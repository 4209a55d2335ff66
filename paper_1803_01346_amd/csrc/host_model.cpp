// Host-side model pieces: scaling of Eq. 8, applied-field drives, voxelizer.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "host_model.h"

namespace scfft {

const double kMu0 = 4.0e-7 * M_PI;

Units make_units(const scfft_material& m) {
  Units u;
  u.jc = m.jc;
  u.l = m.l_char_m;
  u.e0 = m.e0;
  u.t0 = kMu0 * m.jc * m.l_char_m * m.l_char_m / m.e0;  // Eq. 8
  u.h_scale = m.jc * m.l_char_m;
  return u;
}

bool validate_material(const scfft_material& m, const char** why) {
  if (!(m.jc > 0.0) || !std::isfinite(m.jc)) { *why = "jc must be positive"; return false; }
  if (!(m.e0 > 0.0) || !std::isfinite(m.e0)) { *why = "e0 must be positive"; return false; }
  if (!(m.l_char_m > 0.0) || !std::isfinite(m.l_char_m)) { *why = "l_char_m must be positive"; return false; }
  if (!(m.n_power >= 1.0) || !std::isfinite(m.n_power)) { *why = "n_power must be >= 1"; return false; }
  if (!(m.rho_out >= 0.0) || !std::isfinite(m.rho_out)) { *why = "rho_out must be >= 0"; return false; }
  return true;
}

bool Drive::set(const scfft_drive& d, const Units& u, const char** why) {
  kind = d.kind;
  double n = std::sqrt(d.dir[0] * d.dir[0] + d.dir[1] * d.dir[1] + d.dir[2] * d.dir[2]);
  for (int c = 0; c < 3; ++c) dir[c] = n > 0.0 ? d.dir[c] / n : 0.0;
  const double to_h = 1.0 / (kMu0 * u.h_scale);
  amp = d.amp_T * to_h;
  tk.clear();
  bk.clear();
  if (kind == SCFFT_DRIVE_RAMP_HOLD) {
    if (!(d.t_ramp_s > 0.0)) { *why = "t_ramp_s must be positive"; return false; }
    t_ramp = d.t_ramp_s / u.t0;
  } else if (kind == SCFFT_DRIVE_SINE) {
    omega = 2.0 * M_PI * d.freq_hz * u.t0;
  } else if (kind == SCFFT_DRIVE_PWL) {
    if (d.n_pts < 1 || !d.t_s || !d.b_T) { *why = "pwl drive needs n_pts >= 1 points"; return false; }
    for (int k = 0; k < d.n_pts; ++k) {
      if (k > 0 && !(d.t_s[k] > d.t_s[k - 1])) { *why = "pwl times must increase"; return false; }
      tk.push_back(d.t_s[k] / u.t0);
      for (int c = 0; c < 3; ++c) bk.push_back(d.b_T[3 * k + c] * to_h);
    }
  } else {
    *why = "unknown drive kind";
    return false;
  }
  return true;
}

void Drive::eval(double t, double he[3], double hedot[3]) const {
  if (kind == SCFFT_DRIVE_RAMP_HOLD) {
    const double f = t < t_ramp ? t / t_ramp : 1.0;
    const double r = t < t_ramp ? amp / t_ramp : 0.0;
    for (int c = 0; c < 3; ++c) {
      he[c] = dir[c] * amp * f;
      hedot[c] = dir[c] * r;
    }
  } else if (kind == SCFFT_DRIVE_SINE) {
    for (int c = 0; c < 3; ++c) {
      he[c] = dir[c] * amp * std::sin(omega * t);
      hedot[c] = dir[c] * amp * omega * std::cos(omega * t);
    }
  } else {
    const size_t n = tk.size();
    if (n == 0) {
      for (int c = 0; c < 3; ++c) he[c] = hedot[c] = 0.0;
      return;
    }
    if (t < tk[0] || t >= tk[n - 1]) {
      const size_t k = t < tk[0] ? 0 : n - 1;
      for (int c = 0; c < 3; ++c) {
        he[c] = bk[3 * k + c];
        hedot[c] = 0.0;
      }
      return;
    }
    size_t i = 0;
    while (i + 1 < n && tk[i + 1] <= t) ++i;
    const double dt = tk[i + 1] - tk[i];
    for (int c = 0; c < 3; ++c) {
      const double s = (bk[3 * (i + 1) + c] - bk[3 * i + c]) / dt;
      he[c] = bk[3 * i + c] + s * (t - tk[i]);
      hedot[c] = s;
    }
  }
}

std::vector<double> Drive::kinks() const {
  if (kind == SCFFT_DRIVE_RAMP_HOLD) return {t_ramp};
  if (kind == SCFFT_DRIVE_PWL) return tk;
  return {};
}

// Signed margin of a node to a primitive (positive inside), dimensionless.
static double margin(const scfft_shape& s, double inv_l, double x, double y, double z) {
  const double p[3] = {x - s.center_m[0] * inv_l, y - s.center_m[1] * inv_l, z - s.center_m[2] * inv_l};
  if (s.kind == SCFFT_SHAPE_BOX) {
    double g = s.size_m[0] * inv_l - std::fabs(p[0]);
    g = std::fmin(g, s.size_m[1] * inv_l - std::fabs(p[1]));
    return std::fmin(g, s.size_m[2] * inv_l - std::fabs(p[2]));
  }
  if (s.kind == SCFFT_SHAPE_CYLINDER) {
    const int a = s.axis;
    const double u = p[(a + 1) % 3], v = p[(a + 2) % 3];
    const double rho = std::sqrt(u * u + v * v);
    return std::fmin(s.size_m[0] * inv_l - rho, s.size_m[2] * inv_l - std::fabs(p[a]));
  }
  return s.size_m[0] * inv_l - std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
}

bool validate_shapes(const scfft_shape* shapes, int n, const char** why) {
  if (n < 0 || (n > 0 && !shapes)) { *why = "shapes: bad count or NULL"; return false; }
  for (int i = 0; i < n; ++i) {
    const scfft_shape& s = shapes[i];
    if (s.kind < SCFFT_SHAPE_BOX || s.kind > SCFFT_SHAPE_SPHERE) { *why = "shape: unknown kind"; return false; }
    if (s.op != SCFFT_OP_ADD && s.op != SCFFT_OP_SUB) { *why = "shape: unknown op"; return false; }
    if (s.kind == SCFFT_SHAPE_CYLINDER && (s.axis < 0 || s.axis > 2)) { *why = "shape: axis must be 0, 1 or 2"; return false; }
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(s.center_m[c]) || !std::isfinite(s.size_m[c])) { *why = "shape: non-finite value"; return false; }
  }
  return true;
}

void voxelize(const int n[3], const double half_width_dimless[3], double l_m,
              const scfft_shape* shapes, int n_shapes, uint8_t* mask) {
  const int nx = n[0], ny = n[1], nz = n[2];
  double h[3];
  for (int a = 0; a < 3; ++a) h[a] = 2.0 * half_width_dimless[a] / n[a];
  const double eps = 1e-9 * std::fmin(h[0], std::fmin(h[1], h[2]));
  const double inv_l = 1.0 / l_m;
  std::memset(mask, 0, (size_t)nx * ny * nz);
  for (int k = 0; k < nz; ++k) {
    const double z = -half_width_dimless[2] + (k + 0.5) * h[2];
    for (int j = 0; j < ny; ++j) {
      const double y = -half_width_dimless[1] + (j + 0.5) * h[1];
      uint8_t* row = mask + ((size_t)k * ny + j) * nx;
      for (int i = 0; i < nx; ++i) {
        const double x = -half_width_dimless[0] + (i + 0.5) * h[0];
        bool in = false;
        for (int s = 0; s < n_shapes; ++s) {
          const double g = margin(shapes[s], inv_l, x, y, z);
          if (shapes[s].op == SCFFT_OP_ADD) {
            if (g > eps) in = true;
          } else if (g > -eps) {
            in = false;
          }
        }
        row[i] = in ? 1 : 0;
      }
    }
  }
}

// ---- topology of Omega ----------------------------------------------------
// Omega is taken as the union K of the closed voxels of its nodes.  b0 counts
// the components of K (voxels touching at a face, edge or corner connect);
// b2 counts the bounded components of the complement (empty voxels connect
// only through faces, the consistent pairing with the 26-neighbourhood, and
// everything outside the grid belongs to the unbounded one); the Euler
// characteristic chi = V - E + F - C of the cubical complex gives
// b1 = b0 + b2 - chi, the number of independent closed contours in Omega that
// bound no surface inside it.

namespace {

int find_root(std::vector<int32_t>& p, int32_t a) {
  while (p[a] != a) {
    p[a] = p[p[a]];
    a = p[a];
  }
  return a;
}

void unite(std::vector<int32_t>& p, int32_t a, int32_t b) {
  a = find_root(p, a);
  b = find_root(p, b);
  if (a != b) p[std::max(a, b)] = std::min(a, b);
}

// chi contribution of the cells whose lowest corner is the lattice point p,
// indexed by the 2x2x2 block of voxels around p (bit dx + 2 dy + 4 dz for the
// voxel at offset (dx - 1, dy - 1, dz - 1) from p): the vertex p, the three
// edges leaving p upwards, the three faces and the cube with lowest corner p.
// A cell belongs to K when any voxel containing it is filled.
struct ChiTable {
  int8_t v[256];
  ChiTable() {
    for (int c = 0; c < 256; ++c) {
      auto any = [c](int need_x, int need_y, int need_z) {
        for (int b = 0; b < 8; ++b) {
          const int dx = b & 1, dy = (b >> 1) & 1, dz = (b >> 2) & 1;
          if ((need_x && !dx) || (need_y && !dy) || (need_z && !dz)) continue;
          if (c & (1 << b)) return 1;
        }
        return 0;
      };
      v[c] = (int8_t)(any(0, 0, 0) - any(1, 0, 0) - any(0, 1, 0) - any(0, 0, 1) + any(1, 1, 0) +
                      any(1, 0, 1) + any(0, 1, 1) - any(1, 1, 1));
    }
  }
};

}  // namespace

namespace {
void betti_of_box(const int n[3], const uint8_t* mask, int64_t betti[3]);
}

// The numbers depend only on the bounding box of Omega and one empty layer
// around it (everything farther out is empty and joined to the unbounded
// component), so the count runs on that crop of the grid.
void mask_betti(const int n[3], const uint8_t* mask, int64_t betti[3]) {
  int lo[3] = {n[0], n[1], n[2]}, hi[3] = {-1, -1, -1};
  for (int z = 0; z < n[2]; ++z)
    for (int y = 0; y < n[1]; ++y) {
      const uint8_t* row = mask + ((size_t)z * n[1] + y) * n[0];
      for (int x = 0; x < n[0]; ++x)
        if (row[x]) {
          const int id[3] = {x, y, z};
          for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], id[a]);
            hi[a] = std::max(hi[a], id[a]);
          }
        }
    }
  if (hi[0] < 0) {
    betti[0] = betti[1] = betti[2] = 0;
    return;
  }
  int c[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = std::max(0, lo[a] - 1);
    hi[a] = std::min(n[a] - 1, hi[a] + 1);
    c[a] = hi[a] - lo[a] + 1;
  }
  std::vector<uint8_t> crop((size_t)c[0] * c[1] * c[2]);
  for (int z = 0; z < c[2]; ++z)
    for (int y = 0; y < c[1]; ++y)
      std::memcpy(&crop[((size_t)z * c[1] + y) * c[0]],
                  mask + ((size_t)(z + lo[2]) * n[1] + (y + lo[1])) * n[0] + lo[0], (size_t)c[0]);
  betti_of_box(c, crop.data(), betti);
}

namespace {
void betti_of_box(const int n[3], const uint8_t* mask, int64_t betti[3]) {
  const int nx = n[0], ny = n[1], nz = n[2];
  const size_t nodes = (size_t)nx * ny * nz;
  if (nodes >= (size_t)INT32_MAX) {
    betti[0] = betti[1] = betti[2] = -1;
    return;
  }
  auto at = [&](int x, int y, int z) -> int {
    if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return 0;
    return mask[((size_t)z * ny + y) * nx + x] != 0;
  };
  // Euler characteristic
  static const ChiTable table;
  int64_t chi = 0;
  for (int z = 0; z <= nz; ++z)
    for (int y = 0; y <= ny; ++y)
      for (int x = 0; x <= nx; ++x) {
        int c = 0;
        for (int b = 0; b < 8; ++b)
          c |= at(x - 1 + (b & 1), y - 1 + ((b >> 1) & 1), z - 1 + ((b >> 2) & 1)) << b;
        chi += table.v[c];
      }
  // components: one union-find over all voxels plus the outside (index nodes)
  std::vector<int32_t> p(nodes + 1);
  for (size_t i = 0; i <= nodes; ++i) p[i] = (int32_t)i;
  const int32_t outside = (int32_t)nodes;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int32_t i = (int32_t)(((size_t)z * ny + y) * nx + x);
        if (at(x, y, z)) {
          // earlier 26-neighbours (13 of them) of a filled voxel
          for (int dz = -1; dz <= 0; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                if (dz == 0 && (dy > 0 || (dy == 0 && dx >= 0))) continue;
                if (at(x + dx, y + dy, z + dz))
                  unite(p, i, (int32_t)(((size_t)(z + dz) * ny + (y + dy)) * nx + (x + dx)));
              }
        } else {
          if (x == 0 || y == 0 || z == 0 || x == nx - 1 || y == ny - 1 || z == nz - 1) unite(p, i, outside);
          if (x > 0 && !at(x - 1, y, z)) unite(p, i, i - 1);
          if (y > 0 && !at(x, y - 1, z)) unite(p, i, i - nx);
          if (z > 0 && !at(x, y, z - 1)) unite(p, i, i - nx * ny);
        }
      }
  int64_t b0 = 0, b2 = 0;
  const int32_t root_out = find_root(p, outside);
  for (size_t i = 0; i < nodes; ++i)
    if (p[i] == (int32_t)i && (int32_t)i != root_out) (mask[i] ? b0 : b2) += 1;
  betti[0] = b0;
  betti[1] = b0 + b2 - chi;
  betti[2] = b2;
}
}  // namespace

}  // namespace scfft
