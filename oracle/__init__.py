"""Plain, slow FP64 CPU oracle for weighted-quadrature (WQ / DWQ) row assembly.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the package entry
module and the CPU-baseline leg of the benchmark may import this package.  The
product path (the HIP library and its Python binding) never imports, links or calls
anything here, and nothing here imports the product path.

What it computes (Marussig, "Fast formation and assembly for spline-based 3D
fictitious domain methods"):
  * tensor-product B-splines of degree p, maximal smoothness, open uniform knots,
    identity geometry map (Section 2);
  * function types exterior / interior / cut from the overlap of the support with
    the domain (Section 2.1);
  * weighted-quadrature rules per test function and direction (Section 1, WQ
    ingredient; Section 2.2 step 1), with the WQ points chosen among the element
    Gauss points (Section 2.2, last paragraph);
  * discontinuous weighted quadrature for cut functions: split search, knot
    insertion to a C^-1 break, nested points, refined weights, recombination
    through the subdivision matrix (Section 2.2 steps 2-6 and the paragraph after
    Fig. 3), and the domain splitting of Eq. (1);
  * element-wise Gauss integration of the remaining interior elements and of cut
    elements (here: octree sub-cells with a point indicator);
  * mass and stiffness matrices as direct sums over quadrature points, entry by
    entry (no sum factorization), the conventional element-loop Gauss assembly,
    and the adjoint dL/dkappa for L = sum_IJ G_IJ A_IJ.

Readings of points the paper leaves open are listed in the module docstrings where
they are used.  Every function here is pinned by the CPU tests against closed forms,
invariants or brute force.
"""
