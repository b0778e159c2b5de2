// Shared set-up of the TT assembly (assemble.cpp) and of its adjoint (adjoint.cpp): the
// univariate spaces per direction, the quadrature, the interpolation space of the weights
// and the geometry basis tables at its Greville points.
#pragma once

#include <vector>

#include "common.hpp"

namespace iga {

struct SpaceDir {
  int n, N, E, nt;  // free functions, all functions, elements, interpolation-space size
  std::vector<double> ksol, kint, grev, qpts, qw;
  DBuf dksol, dkint, dgrev, dqpts, dqw;
  DBuf Bv, Bd, Bt;  // [Q][N] values, derivatives; [Q][nt] interpolation basis (Q = E nq)
  DBuf Binv;        // [nt][nt]: inverse of the collocation matrix [g][m] = beta~_m(g)
};
// Degree-p solution space with n[d] free functions, interpolation degree pt, nq Gauss
// points per element, for the three directions.
void setup_spaces(iga_ctx* ctx, int p, const int n[3], int pt, int nq, SpaceDir dir[3]);

struct GeometryTables {
  DBuf gk[3], Bv[3], Bd[3], ctrl;  // geometry knots, basis values / derivatives at the Greville points
  const double* bv[3];
  const double* bd[3];
};
void geometry_tables(iga_ctx* ctx, const iga_geometry* geo, const SpaceDir dir[3], GeometryTables& gt);
void check_geometry(const iga_geometry* geo);

}  // namespace iga
