"""Reading and writing two-element EAM tables in the DYNAMO "setfl" text
format, the form in which published alloy EAM potentials (such as Fe-Cu
ones) are commonly distributed, so that they can drive the library through
inputs.EamTable (vcsgc_eam_table).

The format: three comment lines; the element count and names; Nrho, drho,
Nr, dr and the cutoff; per element a line (atomic number, mass, lattice
constant, lattice name) followed by F(rho) at rho_k = k drho (Nrho values)
and f(r) at r_k = k dr (Nr values); then r phi(r) (Nr values) for every
element pair i >= j in the order (1,1), (2,1), (2,2).  Values may wrap over
lines freely.  The pair columns hold r phi(r): phi(r_k) = (r phi)_k / r_k
for k >= 1, and phi(0) is taken as phi(r_1) (no pair is ever at r = 0).
"""
from __future__ import annotations

import numpy as np

from .inputs import EamTable


def read(path: str):
    """Returns (table, elements, masses) of a two-element setfl file."""
    with open(path) as fh:
        lines = fh.read().splitlines()
    head = lines[3].split()
    nel = int(head[0])
    if nel != 2:
        raise ValueError(f"two elements expected, the file has {nel}")
    elements = head[1:1 + nel]
    g = lines[4].split()
    nrho, drho, nr, dr, rc = int(g[0]), float(g[1]), int(g[2]), float(g[3]), float(g[4])
    tokens = " ".join(lines[5:]).split()
    pos = 0

    def take(k):
        nonlocal pos
        v = np.array([float(t) for t in tokens[pos:pos + k]], dtype=np.float64)
        if v.size != k:
            raise ValueError("setfl file ends early")
        pos += k
        return v

    masses, F, f = [], [], []
    for _ in range(nel):
        info = tokens[pos:pos + 4]
        pos += 4
        masses.append(float(info[1]))
        F.append(take(nrho))
        f.append(take(nr))
    r = dr * np.arange(nr, dtype=np.float64)
    phi = []
    for _ in range(nel * (nel + 1) // 2):
        rphi = take(nr)
        p = np.empty(nr)
        p[1:] = rphi[1:] / r[1:]
        p[0] = p[1]
        phi.append(p)
    table = EamTable(rc, dr, drho, np.ascontiguousarray(np.stack(f)),
                     np.ascontiguousarray(np.stack(phi)), np.ascontiguousarray(np.stack(F)))
    return table, elements, masses


def write(path: str, table: EamTable, elements=("A", "B"), masses=(55.845, 63.546),
          numbers=(26, 29), lattice=(2.87, 2.87), comment: str = "") -> None:
    """Writes a two-element table as setfl (r phi in the pair columns), five
    values per line with 17 significant digits, which read() returns bit for
    bit except the pair values, recovered as (r phi) / r."""
    r = table.dr * np.arange(table.nr, dtype=np.float64)

    def block(v):
        v = np.asarray(v, dtype=np.float64)
        return ["  ".join(f"{x:.17g}" for x in v[k:k + 5]) for k in range(0, v.size, 5)]

    out = [comment or "two-element EAM table", "written by paper_1012_5082_amd.setfl", "",
           f"2 {elements[0]} {elements[1]}",
           f"{table.nrho} {table.drho:.17g} {table.nr} {table.dr:.17g} {table.rc:.17g}"]
    for e in range(2):
        out.append(f"{numbers[e]} {masses[e]:.17g} {lattice[e]:.17g} bcc")
        out += block(table.F[e])
        out += block(table.f[e])
    for k in range(3):
        out += block(r * table.phi[k])
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
