"""p-scaling of the preconditioner's patch work with and without the
interior-interface split (fig:complexities; Sec. 6.1 and the complexity
paragraph of Sec. 6: O(p^6) flops and O(p^4) storage for the split
decompositions in 3D, O(p^9) flops and O(p^6) storage without it), counted
on the patches themselves (no GPU).

The decompositions are the figure's: H(grad) PAFW(0)(X^0_Gamma) + J against
PAFW(0)(X^0); H(curl) PH(X^0_Gamma, X^{1,I}_Gamma) + J against PH(X^0,
X^{1,I}) (edge stars and vertex-star potentials); H(div) PAFW(1)(X^2_Gamma)
+ J against PAFW(1)(X^2); Freudenthal mesh with 3 cells per edge, p = 2..8.
Per patch of m columns: storage of the factor (inverse) m(m+1)/2 entries,
setup m^3 flops (Cholesky, triangular inverse and product, m^3/3 each),
2 m^2 flops per application.  The coarse space W^k, the Jacobi group and
the operator are the same with and without the split and are left out.

Checked on the log-log slopes over p = 5..8 (measured: setup 7.21 / 9.56
for H(grad), 7.02 / 9.26 for H(curl), 5.59 / 8.56 for H(div), split /
full; storage 4.78 / 6.30, 4.45 / 6.10, 3.71 / 5.69): without the split
the setup slope is at least 2 larger and the storage slope at least 1.4;
the full forms reach at least 8.5 and 5.5 (the paper's 9 and 6); the split
forms stay within 1.3 of p^6 and 1.0 of p^4 -- the vertex stars of
X^0_Gamma (H(grad), and H(curl)'s potentials) grow like p^2 only once
their face dofs dominate, so at these degrees their exponents sit above
the asymptotic ones; and the split is the cheaper at every p >= 3.  Run
with -s to print the table.
"""
import numpy as np
import pytest

from oracle.element import element
from oracle.mesh import Topology
from oracle.precond import patch_lists, potential_patches
from paper_2506_17406_amd.workloads import kuhn_mesh

P_RANGE = range(2, 9)


def _sizes(top, fam, p, full):
    sizes = [len(x) for x in patch_lists(top, fam, "paper-full" if full else "paper")]
    if fam == "Ned":
        cg_N = (1, p - 1, (p - 1) * (p - 2) // 2, (p - 1) * (p - 2) * (p - 3) // 6)
        sizes += [G.shape[1] for G in potential_patches(top, cg_N, full=full)]
    return np.array(sizes, dtype=float)


def counts():
    X, C = kuhn_mesh(3, 3)
    out = {}
    for fam in ("CG", "Ned", "RT"):
        for p in P_RANGE:
            top = Topology(X, C, element(3, fam, p))
            for full in (False, True):
                m = _sizes(top, fam, p, full)
                out[(fam, p, full)] = dict(n_dofs=top.n_dofs, storage=float((m * (m + 1) / 2).sum()),
                                           setup=float((m ** 3).sum()), apply=float(2 * (m ** 2).sum()),
                                           max=int(m.max()))
    return out


def _slope(c, fam, full, key):
    ps = np.arange(5, 9)
    return np.polyfit(np.log(ps), np.log([c[(fam, p, full)][key] for p in ps]), 1)[0]


@pytest.mark.slow
def test_split_versus_full_patch_scaling():
    c = counts()
    print()
    print("| space | p | dofs | split: max m, factor entries, setup flops, flops/apply | "
          "full: max m, factor entries, setup flops, flops/apply |")
    for fam in ("CG", "Ned", "RT"):
        for p in P_RANGE:
            s, f = c[(fam, p, False)], c[(fam, p, True)]
            print(f"| {fam} | {p} | {s['n_dofs']} | {s['max']}, {s['storage']:.3g}, {s['setup']:.3g}, "
                  f"{s['apply']:.3g} | {f['max']}, {f['storage']:.3g}, {f['setup']:.3g}, {f['apply']:.3g} |")
    for fam in ("CG", "Ned", "RT"):
        ss, sf = _slope(c, fam, False, "setup"), _slope(c, fam, True, "setup")
        ts, tf = _slope(c, fam, False, "storage"), _slope(c, fam, True, "storage")
        print(f"{fam}: setup slopes split {ss:.2f} full {sf:.2f}; storage slopes split {ts:.2f} full {tf:.2f}")
        assert sf - ss >= 2.0 and tf - ts >= 1.4
        assert ss <= 6 + 1.3 and ts <= 4 + 1.0
        assert sf >= 8.5 and tf >= 5.5
        # and the split is the cheaper one at every degree above 2
        for p in range(3, 9):
            assert c[(fam, p, False)]["setup"] <= c[(fam, p, True)]["setup"]
