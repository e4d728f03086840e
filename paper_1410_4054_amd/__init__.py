"""MI355X (gfx950) pipelined CG / BiCGStab with kernel fusion (arXiv:1410.4054).

    from paper_1410_4054_amd import fk, problems
    A = fk.Matrix(problems.poisson3d(128))
    res = fk.solve(A, b_dev, x_dev, method="cg_pipelined", rtol=1e-8)

`fk` is the binding of libfk.so (include/fk.h); `problems` builds the seeded
synthetic inputs.  Importing the package loads nothing: the library is
loaded on the first call into `fk`.
"""
__all__ = ["fk", "problems"]
__version__ = "0.1.0"
