// Host-side model pieces shared by the C-ABI layer.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/scfft.h"

namespace scfft {

extern const double kMu0;

// Eq. 8 scaling.
struct Units {
  double jc, l, e0;
  double t0;       // mu0 jc l^2 / e0
  double h_scale;  // jc l, A/m per unit of h'
};

Units make_units(const scfft_material& m);
bool validate_material(const scfft_material& m, const char** why);

// Applied field in dimensionless units (times t' = t / t0).
struct Drive {
  int kind = SCFFT_DRIVE_RAMP_HOLD;
  double dir[3] = {0.0, 0.0, 1.0};
  double amp = 0.0;
  double t_ramp = 1.0;
  double omega = 0.0;
  std::vector<double> tk, bk;
  bool set(const scfft_drive& d, const Units& u, const char** why);
  // h_e(t') and its right derivative dh_e/dt'
  void eval(double t, double he[3], double hedot[3]) const;
  std::vector<double> kinks() const;
};

bool validate_shapes(const scfft_shape* shapes, int n, const char** why);
// mask[z][y][x] = 1 for nodes of Omega; shapes in metres, scaled by 1/l_m.
void voxelize(const int n[3], const double half_width_dimless[3], double l_m,
              const scfft_shape* shapes, int n_shapes, uint8_t* mask);

// Betti numbers (b0, b1, b2) of the union of the closed voxels of mask
// [Nz][Ny][Nx] (nonzero = Omega), as a subset of R^3; all -1 when the grid
// has 2^31 - 1 nodes or more.
void mask_betti(const int n[3], const uint8_t* mask, int64_t betti[3]);

}  // namespace scfft
