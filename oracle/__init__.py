"""FP64 CPU oracle for MPM-2P on top of MRCM (arXiv 2103.11050).

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct reference that
the HIP path is checked against. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.

It shares no code with the HIP path. It follows the paper's steps in the paper's notation:

* ``fine``       -- lowest-order mixed FEM on rectangles with trapezoidal velocity quadrature,
                    i.e. the two-point flux system, on any block of cells with Dirichlet,
                    Neumann or Robin data on each boundary face (Sections 2-3).
* ``physics``    -- mobilities, conductivity, fractional flow and its derivative
                    (Section 2 and the Corey curves of Section 5).
* ``mrcm``       -- the Multiscale Robin Coupled Method: homogeneous and non-homogeneous
                    basis functions, the interface system, reconstruction (Section 3).
* ``downscale``  -- the local all-Neumann problems that produce a conservative velocity
                    (Section 4.1, the downscaling problems after eq:soma_u).
* ``mpm``        -- the zeroth-order perturbation problem solved with reused basis
                    functions (Section 4.1, eq:mpm_tf_3), optionally with the first-order
                    term (eq:mpm_tf_4, l = 1).
* ``transport``  -- explicit Euler + first-order upwind saturation step (Section 4).
* ``splitting``  -- the modified operator splitting (Section 4.2, Algorithm 1).
* ``cost``       -- basis-function counts and the Relative Cost Reduction (Section 4.3).

Where the paper is silent the oracle takes the readings listed in the design notes of the
repository (fine element, orientation, epsilon norm, switch timing, downscaling of MRCM,
discrete form of kappa^n grad p^m, transport time step, breakthrough).

Parity status: every function here is pinned by a ``-m "not gpu"`` test. The MRCM solution
with interface elements longer than one fine face (constant and linear spaces) is pinned by a
monolithic assembly of the whole system written face by face, with no basis functions; the
MPM-2P velocity (zeroth and first order) on such decompositions by the same assembly applied
to the perturbation problems, followed by the downscaling. The first-order term is also pinned
where MRCM is exact (second Richardson step, error cubic in the perturbation) and by vanishing
without perturbation.
"""
