"""Seeded initial parameters of the learned preconditioner network.

The flat float32 layout is the one documented with the network (8 -> 64 -> 64
-> 64 message-passing layers, then the preconditioner and initial-guess
heads).  The heads start near the Jacobi preconditioner and a Jacobi-scaled
initial guess: delta = softplus(c_d) = 1, p = softplus(c_p) small, rho = 0,
gamma = c_g = 1, eta = 0.
"""

from __future__ import annotations

import math

import numpy as np

F_IN, HID = 8, 64
SIZES = [("W1s", HID * F_IN), ("W1n", HID * F_IN), ("b1", HID),
         ("W2s", HID * HID), ("W2n", HID * HID), ("b2", HID),
         ("W3s", HID * HID), ("W3n", HID * HID), ("b3", HID),
         ("a_d", HID), ("c_d", 1), ("a_g", HID), ("c_g", 1),
         ("a_p1", HID), ("a_p2", HID), ("c_p", 1), ("a_r", HID), ("c_r", 1), ("a_e", HID), ("c_e", 1)]
N_PARAMS = sum(n for _, n in SIZES)


def init_params(seed: int = 0, head_scale: float = 0.01) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = []
    for name, n in SIZES:
        if name.startswith("W"):
            fan_in = F_IN if name.startswith("W1") else HID
            out.append(rng.standard_normal(n) * math.sqrt(1.0 / fan_in))
        elif name.startswith("a_"):
            out.append(rng.standard_normal(n) * head_scale)
        elif name == "c_d":
            out.append(np.array([math.log(math.e - 1.0)]))
        elif name == "c_g":
            out.append(np.array([1.0]))
        elif name == "c_p":
            out.append(np.array([-4.0]))
        else:
            out.append(np.zeros(n))
    return np.concatenate(out).astype(np.float32)
