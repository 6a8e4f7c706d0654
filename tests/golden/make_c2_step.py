"""Writes the expected values of the 40 x 10 x 10 cantilever check (rest-position parameters, seed 0).

Every value comes from the FP64 oracle (oracle/dense.py): the frozen length scale and the surface
targets of the problem set-up, the equilibrium x(p0) (Newton with dense Cholesky, |c| <= 1e-11 |f|),
the dense Gauss-Newton step at (x(p0), p0) with its three blocks (S = -Kx^-1 Kp, H = S^T A S + C,
H dp = -g, dx = S dp, dlam from eq. GNdlambda), and the same step refined in the saddle-point system
with extended-precision residuals (polish_sgn_solution; the explicit H rounds the dense step at
about 4e-9 relative in dp at this size, the refined step is the saddle-point solution to about 1e-12).
The dense step needs about 2e13 flops and 12 GB, a few minutes on host cores, so the GPU test reads
the values from this file instead of recomputing them.

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
    t = time.time()
    b = D.sgn_rhs(prob, x, p)
    z, hist = D.polish_sgn_solution(prob, x, p, np.concatenate([st.dx, st.dp, st.dlam]), b, sweeps=2)
    print(f"refined step {time.time() - t:.0f} s, equilibrated residuals " + " ".join(f"{h:.2e}" for h in hist),
          flush=True)
    nx, npar = prob.n_x, prob.n_p
    np.savez_compressed(OUT, length_scale=prob.length_scale, target_val=prob.target_val, x_eq=x,
                        dx=st.dx, dp=st.dp, dlam=st.dlam, grad=st.grad,
                        ref_dx=z[:nx], ref_dp=z[nx:nx + npar], ref_dlam=z[nx + npar:])
    print("wrote", OUT)


if __name__ == "__main__":
    main()
