"""Plain FP64 CPU reference for the boundary-condition operator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_2605_14780_amd``) never imports, calls or links anything here,
and this package imports nothing from it: the two share no code.  The only
module both sides use is ``synthinputs`` (seeded input arrays, no operator
arithmetic).

What it computes (Mat2Boundary, arXiv 2605.14780):

* ``grid``          the region model: global box, blocks as full/data slices
                    (start, stop, step: the points start + k step < stop) with
                    the block id as leading coordinate, ghost = full - data
                    (Sec. III-A; Sec. IV-A-1; Alg. 1 region lines).
* ``operator``      assembly of the affine operator F(x) = A x + b over the
                    ghost rows from basic sub-matrices / sub-vectors, applied
                    in place on a full field; its vector-Jacobian product
                    (Sec. III-B; Sec. IV-A-3/4, Tables II and III).
* ``cubed_sphere``  the equiangular gnomonic cubed sphere: face-edge halo
                    copy with rotated axes and 4-point Lagrange rows along the
                    neighbour's grid line, built from 3-D geometry
                    (Sec. II-B; Sec. III-B user-defined interpolation;
                    Sec. V-A multi-component vectors).
* ``hpcg``          the HPCG-shaped Cartesian case: 2x2x2 blocks with halo 1,
                    halo copy between blocks, zero padding outside, then the
                    27-point operator (Sec. III-B halo copying and zero
                    padding; Sec. IV-C, BC writes feed the inner operator).
* ``dense``         brute-force dense A on tiny grids, evaluated entry by entry
                    from the definitions without the sparse assembly.
* ``quadrature``    wide interpolation rows, Sec. III-B's Agg . Recons: a
                    Gauss rule over each ghost cell of tensor-product cubic
                    reconstructions on the neighbour face.
* ``footprint``     the consumer footprint of Sec. IV-C: ghost rows that no
                    read of the consuming operator reaches, and the operator
                    restricted to the others.
* ``consumer``      the operator that reads the BC's ghosts (Sec. IV-C): a
                    stencil of offsets and weights on the field the BC has
                    written, the BC applied first, then the shifted sums.
* ``averaging``     block-edge averaging of co-located points (data rows,
                    Sec. III-B), on a vertex-centred cubed sphere, sets found
                    by 3-D position; applied together with the ghost rows, all
                    rows reading the input field.

Pins (in ``tests/test_oracle_*.py``, run with ``-m "not gpu"``) tie each part
to something other than itself: ``numpy.pad`` for zero/circular/symmetric
maps, the Alg. 1 rotated map, cubic reproduction and fourth-order convergence
of the Lagrange rows, a solid-body-rotation vector field for the component
rotation, the closed form of the 27-point operator on a constant field, the
dot-product identity for the adjoint, and the cube's vertex count and
edge/corner sharing for the averaging sets.
"""
from .grid import Grid, Box  # noqa: F401
from .operator import (  # noqa: F401
    MapSub, ZeroSub, RowsSub, VectorSub, Operator, assemble, apply, vjp,
)
