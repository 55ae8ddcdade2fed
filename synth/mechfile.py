"""Plain-text mechanism file ("dfmech 1"), reader and writer.

The format is keyword-driven and fully numeric apart from names, so that a
C reader needs nothing beyond ``fscanf``.  Every section is introduced by its
keyword and followed by a fixed number of whitespace-separated values whose
count follows from ``n_elements`` (E), ``n_species`` (K) and ``n_reactions``
(M).  Lines starting with ``#`` are comments.

Sections, in order::

    dfmech 1
    name <token>
    seed <int>
    n_elements E
    n_species K
    n_reactions M
    elements <E names>
    element_mass <E reals, g/mol>
    species <K names>
    molar_mass <K reals, g/mol>
    composition <K rows x E ints>            atoms of element e in species k
    nasa7 <K rows x 7 reals>                 single-range NASA-7 a1..a7
    reaction_type <M ints>                   0 elementary, 1 third body (+M),
                                             2 Troe falloff (+M)
    nu_reac <M rows x K ints>                reactant coefficients nu'
    nu_prod <M rows x K ints>                product coefficients nu''
    arrhenius <M rows x 3 reals>             A [cm-mol-s], b, Ta = Ea/R [K]
                                             (for Troe: the high-pressure k_inf)
    efficiency <M rows x K reals>            third-body efficiencies (1 default)
    falloff_low <M rows x 3 reals>           A0, b0, Ta0 of k_0 (Troe rows only)
    troe <M rows x 4 reals>                  alpha, T***, T*, T** (Troe rows only)
    end

Units: A in (cm^3/mol)^(n-1)/s with n the molecularity counting M, so that
rates are evaluated with concentrations in mol/cm^3.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class Mechanism:
    name: str
    seed: int
    elements: list
    element_mass: np.ndarray          # [E] g/mol
    species: list
    molar_mass: np.ndarray            # [K] g/mol
    composition: np.ndarray           # [K, E] int
    nasa7: np.ndarray                 # [K, 7]
    reaction_type: np.ndarray         # [M] int
    nu_reac: np.ndarray               # [M, K] int
    nu_prod: np.ndarray               # [M, K] int
    arrhenius: np.ndarray             # [M, 3]
    efficiency: np.ndarray            # [M, K]
    falloff_low: np.ndarray           # [M, 3]
    troe: np.ndarray                  # [M, 4]
    meta: dict = field(default_factory=dict)

    @property
    def n_species(self) -> int:
        return len(self.species)

    @property
    def n_reactions(self) -> int:
        return int(self.reaction_type.shape[0])

    @property
    def n_elements(self) -> int:
        return len(self.elements)

    def index(self, name: str) -> int:
        return self.species.index(name)

    def reaction_string(self, j: int) -> str:
        def side(nu):
            parts = []
            for k in range(self.n_species):
                c = int(nu[k])
                if c:
                    parts.append((f"{c} " if c > 1 else "") + self.species[k])
            return " + ".join(parts)
        t = int(self.reaction_type[j])
        m = {0: "", 1: " + M", 2: " (+M)"}[t]
        return f"{side(self.nu_reac[j])}{m} <=> {side(self.nu_prod[j])}{m}"


def _fmt(x) -> str:
    return repr(float(x))


def write_mech(path, mech: Mechanism, header: str = "") -> None:
    K, M, E = mech.n_species, mech.n_reactions, mech.n_elements
    out = []
    for line in header.splitlines():
        out.append("# " + line)
    for j in range(M):
        out.append(f"# R{j:03d}: {mech.reaction_string(j)}")
    out.append("dfmech 1")
    out.append(f"name {mech.name}")
    out.append(f"seed {int(mech.seed)}")
    out.append(f"n_elements {E}")
    out.append(f"n_species {K}")
    out.append(f"n_reactions {M}")
    out.append("elements " + " ".join(mech.elements))
    out.append("element_mass " + " ".join(_fmt(v) for v in mech.element_mass))
    out.append("species " + " ".join(mech.species))
    out.append("molar_mass " + " ".join(_fmt(v) for v in mech.molar_mass))
    out.append("composition")
    for k in range(K):
        out.append(" ".join(str(int(v)) for v in mech.composition[k]))
    out.append("nasa7")
    for k in range(K):
        out.append(" ".join(_fmt(v) for v in mech.nasa7[k]))
    out.append("reaction_type " + " ".join(str(int(v)) for v in mech.reaction_type))
    for key, arr, ints in (("nu_reac", mech.nu_reac, True), ("nu_prod", mech.nu_prod, True),
                           ("arrhenius", mech.arrhenius, False), ("efficiency", mech.efficiency, False),
                           ("falloff_low", mech.falloff_low, False), ("troe", mech.troe, False)):
        out.append(key)
        for j in range(M):
            out.append(" ".join(str(int(v)) if ints else _fmt(v) for v in arr[j]))
    out.append("end")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")


def read_mech(path) -> Mechanism:
    toks = []
    with open(path) as f:
        for line in f:
            s = line.strip()
            if not s or s.startswith("#"):
                continue
            toks.extend(s.split())
    it = iter(toks)

    def nxt():
        return next(it)

    def expect(key):
        t = nxt()
        if t != key:
            raise ValueError(f"{path}: expected '{key}', found '{t}'")

    expect("dfmech")
    if nxt() != "1":
        raise ValueError("unsupported dfmech version")
    expect("name"); name = nxt()
    expect("seed"); seed = int(nxt())
    expect("n_elements"); E = int(nxt())
    expect("n_species"); K = int(nxt())
    expect("n_reactions"); M = int(nxt())
    expect("elements"); elements = [nxt() for _ in range(E)]
    expect("element_mass"); emass = np.array([float(nxt()) for _ in range(E)])
    expect("species"); species = [nxt() for _ in range(K)]
    expect("molar_mass"); W = np.array([float(nxt()) for _ in range(K)])

    def block(key, rows, cols, dtype):
        expect(key)
        return np.array([dtype(nxt()) for _ in range(rows * cols)], dtype=dtype).reshape(rows, cols)

    comp = block("composition", K, E, int)
    nasa = block("nasa7", K, 7, float)
    expect("reaction_type"); rtype = np.array([int(nxt()) for _ in range(M)], dtype=int)
    nu_r = block("nu_reac", M, K, int)
    nu_p = block("nu_prod", M, K, int)
    arr = block("arrhenius", M, 3, float)
    eff = block("efficiency", M, K, float)
    low = block("falloff_low", M, 3, float)
    troe = block("troe", M, 4, float)
    expect("end")
    return Mechanism(name, seed, elements, emass, species, W, comp, nasa, rtype, nu_r, nu_p,
                     arr, eff, low, troe)
