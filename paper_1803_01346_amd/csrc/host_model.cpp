// Host-side model pieces: scaling of Eq. 8, applied-field drives, voxelizer.
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

}  // namespace scfft
