"""Coefficient tables (the model bank).

Each JSON file holds one trained recursion: family, number of layers L, the
training point (beta0, mu0), an optional entropy rescale alpha, the L x 4
table theta[i] = (a_i, b_i, c_i, d_i) of Eq. (mlsp2), and its provenance.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))


@dataclass
class Model:
    name: str
    L: int
    beta0: float
    mu0: float
    theta: np.ndarray
    family: str = "mlsp2"
    kind: str = "fermi"
    alpha: float = 1.0
    meta: dict = field(default_factory=dict)


def path(name: str) -> str:
    return os.path.join(_DIR, name if name.endswith(".json") else name + ".json")


def load(name: str) -> Model:
    with open(path(name)) as f:
        d = json.load(f)
    th = np.asarray(d["theta"], dtype=np.float64)
    return Model(name=os.path.basename(name).replace(".json", ""), L=int(d["L"]),
                 beta0=float(d["beta0"]), mu0=float(d["mu0"]), theta=th,
                 family=d.get("family", "mlsp2"), kind=d.get("kind", "fermi"),
                 alpha=float(d.get("alpha", 1.0)), meta=d)


def save(model: Model, name: str, provenance: str, extra: dict | None = None) -> str:
    d = {"family": model.family, "kind": model.kind, "L": model.L, "beta0": model.beta0,
         "mu0": model.mu0, "alpha": model.alpha, "provenance": provenance}
    if extra:
        d.update(extra)
    lines = ["{"] + [f" {json.dumps(k)}: {json.dumps(v)}," for k, v in d.items()]
    rows = ["  [" + ", ".join(repr(float(v)) for v in r) + "]" for r in model.theta]
    lines.append(' "theta": [')
    lines.append(",\n".join(rows))
    lines.append(" ]")
    lines.append("}")
    p = path(name)
    with open(p, "w") as f:
        f.write("\n".join(lines) + "\n")
    return p


def available():
    return sorted(f[:-5] for f in os.listdir(_DIR) if f.endswith(".json"))
