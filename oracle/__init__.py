"""Oracle: a plain, slow, FP64 CPU implementation of restricted additive Schwarz.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the serving loop) may import, call or link anything here; only
the tests, the smoke check and the bench's CPU-baseline leg use it.  It shares
no code with the HIP path: it is written from the paper (Nayak, Cojean, Anzt,
"Evaluating Abstract Asynchronous Schwarz solvers", arXiv 2003.05361) and from
textbook definitions, with numpy/scipy primitives as single steps.

Modules
  partition  -- owned sets: regular-1d/2d/3d (Sec. 3.2.1) and seeded recursive
                coordinate bisection standing in for the edge-cut partitioner.
  overlap    -- overlapping index sets by breadth-first layers (Sec. 2.1, Fig. 1).
  residual   -- the outer residual b - A x in compensated float64 (Dot2 of
                Ogita, Rump and Oishi): the convergence measure of Sec. 3.3.2.
  local      -- local subdomain matrices and solvers: banded Cholesky factor
                once, triangular solves per iteration (Sec. 3.3.1); fixed-k CG;
                reduced-precision variants.
  schwarz    -- synchronous RAS (Sec. 2.1, Alg. 1), restricted multiplicative
                Schwarz (ordered in-place variant), a seeded asynchronous
                simulator with centralized / decentralized detection (Sec. 2.2,
                Sec. 3.3.2), direct reference solutions.

Parity status: every function here is pinned by a CPU test against the
mathematics (direct solves, block Jacobi, closed-form eigenmodes, the dense
iteration operator, brute-force index sets, textbook CG / Cholesky facts),
except the asynchronous trajectory, which is nondeterministic by design
(Sec. 2.1): its *final result* is pinned (verified residual and error against
the direct solve) but the trajectory itself is "parity unpinned".
"""
from . import partition, overlap, residual, local, schwarz  # noqa: F401
