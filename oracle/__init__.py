"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 implementation of what the Newton-step solve computes,
written from the paper (Tuma, Rezaee-Hajidehi, Hron, Farrell, Stupkiewicz,
"Phase-field modeling of multivariant martensitic transformation at
finite-strain: computational aspects and large-scale finite-element
simulations", CMAME 2021).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path (the HIP
library and its binding) never imports, links or calls anything here, and this
package never imports the product path.

Modules
-------
material  transformation stretches (Sec. 4.1), stiffness tensors (Table 1)
energy    local free energy + dissipation + penalty density (Sec. 2.2, 2.3,
          3.1, 3.2); derivatives come from PyTorch automatic differentiation,
          as the paper obtains them from UFL's (Sec. 3.4)
fem       Q1 hex meshes, element integrals, global residual and tangent as
          first and second derivatives of the discrete potential (Sec. 3.3-3.4)
contact   frictionless penalty contact with a rigid spherical indenter and
          the indentation load (Sec. 2.4, Eqs. Ngap and PenPot)
solver    sparse assembly, Dirichlet lifting, point-block Jacobi, geometric
          multigrid V-cycle, FGMRES, Newton, the indentation driver with
          adaptive time steps (Sec. 3.4)

Parity status: every function is pinned by a CPU test (``tests/test_oracle_*``)
except the end-to-end indentation physics on the synthetic workloads, which is
"parity unpinned": the paper prints no values for them.
"""
