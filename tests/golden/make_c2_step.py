"""Writes the expected values of the 40 x 10 x 10 cantilever check (rest-position parameters, seed 0).

Every value comes from the FP64 oracle (oracle/dense.py): the frozen length scale and the surface
targets of the problem set-up, the equilibrium x(p0) (Newton with dense Cholesky, |c| <= 1e-11 |f|),
and the dense Gauss-Newton step at (x(p0), p0) with its three blocks (S = -Kx^-1 Kp, H = S^T A S + C,
H dp = -g, dx = S dp, dlam from eq. GNdlambda).  The dense step needs about 2e13 flops and 12 GB, a
few minutes on host cores, so the GPU test reads it from this file instead of recomputing it.

    python tests/golden/make_c2_step.py      # writes tests/golden/cantilever_40x10x10_s0_step.npz
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import sgn_inputs as si  # noqa: E402
from oracle import dense as D  # noqa: E402

OUT = os.path.join(HERE, "cantilever_40x10x10_s0_step.npz")


def main():
    t = time.time()
    prob = D.setup_targets(si.config_cantilever_small(0))
    p = prob.p_init()
    x, info = D.equilibrium(prob, p, rtol=1e-11)
    assert info.converged, info
    print(f"set-up and equilibrium {time.time() - t:.0f} s ({info.iters} Newton iterations)", flush=True)
    t = time.time()
    st = D.dense_gn_step(prob, x, p)
    print(f"dense GN step {time.time() - t:.0f} s", flush=True)
    np.savez_compressed(OUT, length_scale=prob.length_scale, target_val=prob.target_val, x_eq=x,
                        dx=st.dx, dp=st.dp, dlam=st.dlam, grad=st.grad)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
