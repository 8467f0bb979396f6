"""Write the oracle's gradient of the bubble-trajectory loss for the adjoint column.

Calls only the CPU oracle (FP64). Loss L(theta) = sum over steps n = 1..N and bubbles b of
|x_b^n(theta) - x_b^n(theta_target)|^2 with theta = (drag_scale, lift_scale, omega); the gradient
is the central difference with step h = 1e-3 in each component, at theta0.

    python tests/golden/make_adjoint_golden.py [--steps 2000] [--threads 8]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def trajectory(w, theta, steps, threads):
    sD, sL, omega = theta
    lat = O.Lattice(*w.shape, omega, w.bc)
    bub = O.Bubbles(pos=w.pos.copy(), d=w.d.copy())
    p = dict(w.params)
    p.update(drag_scale=sD, lift_scale=sL)
    return O.run(lat, O.bubble_params(**p), bub, steps, record=True, nthreads=threads)


def gradient(w, steps, threads, h=1e-3):
    target = trajectory(w, w.meta["target"], steps, threads)
    theta0 = np.array(w.meta["theta0"], dtype=np.float64)
    loss = lambda th: float(np.sum((trajectory(w, th, steps, threads) - target) ** 2))
    L0 = loss(theta0)
    g = np.zeros(3)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        g[i] = (loss(theta0 + e) - loss(theta0 - e)) / (2 * h)
    return L0, g


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "adjoint_64x64x192_oracle_gradient.json"))
    args = ap.parse_args()
    w = W.adjoint(steps=args.steps)
    t0 = time.time()
    L0, g = gradient(w, args.steps, args.threads)
    out = {"workload": w.name, "steps": args.steps, "theta0": list(w.meta["theta0"]),
           "target": list(w.meta["target"]), "h": 1e-3, "loss": L0, "gradient": g.tolist(),
           "parameters": ["drag_scale", "lift_scale", "omega"],
           "seconds": time.time() - t0,
           "command": "python tests/golden/make_adjoint_golden.py --steps %d" % args.steps}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
