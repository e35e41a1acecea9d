"""CPU FP64 oracle for the shallow-moment-equation (SME) time step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2601_04826_amd``) never does, and the two share no code.

Contents
--------
tensors   exact rational basis tensors M, A, B, K (Python ``fractions``)
mesh      generic cell/face lists for 1D, 2D structured and triangle meshes
sme       ctypes driver around ``sme_oracle.c`` (flux, NC matrix, step, CFL)
stoker    exact Riemann solution of the wet dam break (level-0 pin)
mlp       FP64 MLP forward/backward/Adam for the learned closure
lift      3D lifting of a state (sigma levels: z, u, v, w, p)
vam       non-hydrostatic VAM predictor-corrector step in 1D (numpy, sparse solve)
"""
