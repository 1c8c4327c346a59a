"""Seeded synthetic inputs shared by the oracle and the GPU library's tests.

This package only *describes* problems: macro-meshes (map kind + parameters and
face connectivity), octree refinement, per-element polynomial degrees,
coefficient and manufactured-solution descriptors (ids + parameters), and
seeded random vectors.  It holds none of the method's arithmetic: no basis
functions, quadrature, geometry/Jacobians, operators or solvers.  Both the
oracle and the HIP library interpret these descriptions with their own code.

Conventions (the neutral mesh format, documented once here):

* A macro-element is the image of the reference cube [-1,1]^3 under an
  analytic map (the paper's macro-mesh, Sec. II.A.1).  ``macro_kind``:
  0 = AFFINE      x = o + sum_i (xi_i + 1)/2 * a_i; params = o(3), a0(3), a1(3), a2(3)
  1 = SHELL       cubed-sphere shell patch; params[0:9] = R (3x3 row-major signed
                  permutation, det +1), params[9] = radial kind (0 linear,
                  1 inverse, 2 piecewise linear/inverse), params[10] = r_in,
                  params[11] = r_out, params[12] = zeta_break, params[13] = r_break.
                  Direction v = R (tan(pi xi0/4), tan(pi xi1/4), 1); x = r(xi2) v/|v|.
  2 = CUBE_SPHERE wedge between the face of a central cube of half-width
                  ``params[10]`` and the sphere of radius ``params[11]``, in the same
                  angular frame R: the linear blend in xi2 of the flat point
                  a R (xi0, xi1, 1) (parametrised linearly, like the affine cube) and
                  the sphere point along the equiangular direction.
* Faces of the reference cube: f = 2*d + s, normal axis d, s = 0 at xi_d = -1,
  s = 1 at xi_d = +1.  Face coordinates (a, b) are the two tangential reference
  coordinates in increasing axis order.
* Orientation code o (0..7) maps face coordinates (a, b) of one macro face to the
  neighbour's face coordinates (a', b'): (s, t) = (b, a) if o & 1 else (a, b);
  a' = -s if o & 2 else s; b' = -t if o & 4 else t.
* Elements: (macro, level, anchor[3], p) with 0 <= anchor < 2**level; the cell
  covers reference coordinates [-1 + 2 anchor / 2**level, -1 + 2 (anchor+1) / 2**level]
  of its macro.  The order of the element arrays defines the vector layout.
* Boundary condition kinds: 0 interior, 1 Dirichlet, 2 Neumann, 3 Robin.
"""
from .forest import Forest, orient_map_int, face_corner_orientation  # noqa: F401
from .meshes import (  # noqa: F401
    unit_cube, box_grid, uniform_box, cubed_sphere_shell, hp_sphere_cube, puncture_mesh, star_mesh,
    mesh_summary, adapt,
)
from .problems import (  # noqa: F401
    problem_config1, problem_config2, problem_config3, random_vector,
    dof_count, polynomial_problem, gaussian_problem, polynomial_dirichlet_problem,
    puncture_problem, quadratic_nonlinear_problem, star_problem,
)
