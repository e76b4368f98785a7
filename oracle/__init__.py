"""FP64 CPU oracle of the matrix-free Levenberg-Marquardt ptychography method.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously correct
reference that the GPU library is checked against.  Only the test-suite, the
smoke entry point and the CPU-baseline leg of the benchmark may import it; the
product path never does and fails loudly without its compiled library.

It shares no code with the GPU path (no kernels, headers, tables or helpers);
both take their inputs from the ``synth`` module, which holds none of the
method's arithmetic.

Modules
-------
``ptycho``  forward model, error metrics, gradient, JVP/VJP, GGN-vector
            product, the paper's approximate GGN diagonal and the exact one.
``solver``  truncated preconditioned CG and the LM outer loop.
``cnn``     FP64 reference of the small convolutional preconditioner network.

Parity status of each function is stated in its docstring ("pinned by ..."
or "parity unpinned").
"""
from . import ptycho, solver  # noqa: F401
