"""CPU oracle for 3D geometric moments -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, exact reference that the GPU implementation is
checked against.  It follows the definitions of Diggin & Diggin, "Fast 3D Image
Moments" (arXiv 2012.08099): the 3D moment generating sum (Section 1, eq. 2), the
2D moment sum (eq. 1) and the discrete projection images (Section 3.1, eqs. 4-9 and
the further aligned projections listed after eq. 9).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in here.  The product library never does,
and the oracle imports nothing from the product.
"""
from .moments import (  # noqa: F401
    moment_index,
    moment_list,
    moments_bruteforce,
    moments_exact,
    moment_single,
    projection_image,
    image_moments_2d,
    central_moments,
    central_from_raw,
    features,
)
from .paper import (  # noqa: F401
    DRT_DIRS,
    drt_integrals,
    moments_2d_from_integrals,
    n_paper_images,
    paper_images,
    paper_moments,
)
