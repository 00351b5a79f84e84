"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct numpy implementations of what the GPU library
computes, written from the paper (arXiv 2509.22462, "Nonlinear Optimization
with GPU-Accelerated Neural Network Constraints"):

* ``oracle.nn``  — the network predictor (Eq. 3), the reduced-space residual
  g = y - NN(x) (Eq. 5 and Section 3.2.1), its Jacobian, and the Hessian of
  the Lagrangian term sum_i lambda_i Hess NN_i(x) (Eq. 6, Section 3.2.1),
  the latter three independent ways;
* ``oracle.mlp`` — the warm-start MLP's forward pass, MSE loss, backprop and
  Adam step (Adam is the optimizer the paper names in Section 4.2).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product path never does, and this
package imports nothing from the GPU package: the two share no code.
"""
