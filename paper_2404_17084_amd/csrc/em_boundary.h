// The winding weight of a particle that lies on the boundary of a cell.
//
// The integration kernels use the far-field-subtracted form of the pyramid
// sum: the solid-angle parts of all of a cell's pyramids add up to the
// fraction of directions around the particle that point into the cell, and
// that fraction is taken as 1 for a particle inside the cell and 0 outside.
// The walls whose plane holds the particle (distance 0) then enter with the
// planar angle their polygon subtends at the particle.  This is exact in the
// interior and on a wall (the wall's half turn makes up the missing half),
// but not where two or more wall planes meet at the particle, on an edge or
// a vertex of the cell: there the fraction is the dihedral angle over 2 pi,
// or the corner's solid angle over 4 pi.  For such a particle the kernels use
// cell_winding below instead: the signed sum over all walls of the solid
// angle of their triangles (Van Oosterom-Strackee form of the right
// triangle), which the direct form of the pyramid sum implies.
#pragma once

#include <cmath>
#include <cstdint>

#include "em_internal.h"

namespace em {

// Signed solid angle of the right triangle (f, g, v) of a wall seen from a
// particle at distance r0 from the wall's plane, R0 = |f g|, l the signed
// coordinate of v from g along the edge (any common length unit); for
// r0 = 0 the planar angle of the triangle at f.
__device__ __forceinline__ double tri_solid_angle(double r0, double R0, double l)
{
    const double al = fabs(l);
    const double R02 = R0 * R0;
    const double S = sqrt(r0 * r0 + R02 + l * l);
    const double om = atan2(al * R0 * (R02 + l * l), (S + r0) * (R02 * S + r0 * l * l));
    return l < 0.0 ? -om : om;
}

// Fraction of the directions around a particle in the closed cell that point
// into the cell: sum over walls of sigma_j times the wall's signed solid angle
// (sum over its edges of sign(rho) [Omega(l_b) - Omega(l_a)]), over 4 pi.
__device__ __forceinline__ double cell_winding(double px, double py, double pz, int64_t cell,
                                            const int64_t *__restrict__ cfo, const int64_t *__restrict__ fvo,
                                            const double *__restrict__ plane, const EdgeRec *__restrict__ edges)
{
    double sum = 0.0;
    for (int64_t j = cfo[cell]; j < cfo[cell + 1]; j++) {
        const double d = plane[4 * j + 3] - (plane[4 * j] * px + plane[4 * j + 1] * py + plane[4 * j + 2] * pz);
        const double r0 = fabs(d);
        double face = 0.0;
        for (int64_t s = fvo[j]; s < fvo[j + 1]; s++) {
            const EdgeRec E = edges[s];
            const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
            const double rho = E.mx * wx + E.my * wy + E.mz * wz;
            if (rho == 0.0) continue;
            const double la = -(E.ex * wx + E.ey * wy + E.ez * wz);
            const double lb = la + E.L;
            const double t = tri_solid_angle(r0, fabs(rho), lb) - tri_solid_angle(r0, fabs(rho), la);
            face += rho > 0.0 ? t : -t;
        }
        sum += d >= 0.0 ? face : -face;
    }
    return sum * (0.25 * 0.318309886183790671537767526745);
}

// The indicator term of a pair: 0 outside the closed cell; inside it, 1
// unless two or more wall planes hold the particle.
__device__ __forceinline__ double winding_term(bool inside, int n_on, double px, double py, double pz, int64_t cell,
                                               const int64_t *__restrict__ cfo, const int64_t *__restrict__ fvo,
                                               const double *__restrict__ plane, const EdgeRec *__restrict__ edges)
{
    if (!inside) return 0.0;
    if (n_on < 2) return 1.0;
    return cell_winding(px, py, pz, cell, cfo, fvo, plane, edges);
}

}  // namespace em
