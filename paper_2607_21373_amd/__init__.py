"""MI355X (gfx950) implementation of the matrix-free RTO posterior sampler for
3D photoacoustic tomography ("3D Uncertainty Quantification for
Photoacoustic Tomography", arXiv 2607.21373).

The compute path is libpat.so (HIP kernels behind the C ABI of
``include/pat.h``); ``paper_2607_21373_amd.pat`` is its Python binding.
"""
from .pat import (PAT_F32, PAT_F64, PatError, Problem, pat_adjoint, pat_forward,  # noqa: F401
                  pat_host_assemble, pat_prior_apply, pat_problem_create, rto_sample, version)
