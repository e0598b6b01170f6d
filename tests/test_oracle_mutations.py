"""The oracle's pins against planted mistakes: each case copies pf_oracle.c, plants one
plausible mistake (a wrong sign, index, term, weight or transposed operand), builds the
copy with the oracle's flags and runs the pin suite (tests/test_oracle.py) against it in a
fresh process.  Every planted mistake must make some pin fail; the unchanged copy, built
the same way, must pass them all.  CPU only."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "pf_oracle.c")
PINS = os.path.join(HERE, "test_oracle.py")
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-w"]

# (what is wrong, text of pf_oracle.c, the mistaken text)
MUTATIONS = [
    ("permutation sign reversed (Leibniz)",
     "if (p[a] > p[b]) s = -s;", "if (p[a] < p[b]) s = -s;"),
    ("inverse written transposed",
     "AT(inv, n, r, c) = (double)m[r][n + c];", "AT(inv, n, c, r) = (double)m[r][n + c];"),
    ("page transpose copies instead",
     "AT(tk, cols, c, r) = AT(ak, rows, r, c);", "AT(tk, rows, r, c) = AT(ak, rows, r, c);"),
    ("product reads B transposed",
     "double bv = transB ? AT(bk, n, j, p) : AT(bk, kk, p, j);",
     "double bv = transB ? AT(bk, n, j, p) : AT(bk, kk, j % kk, p % n);"),
    ("P1 gradients with the transposed inverse Jacobian",
     "double dphi[12]; /* tjac^{-1} * dshape : dim x nlb */\n        for (int r = 0; r < dim; r++)\n"
     "            for (int j = 0; j < nlb; j++) {\n                double acc = 0.0;\n"
     "                for (int p = 0; p < dim; p++) acc += AT(tinv, dim, r, p) * AT(ds, dim, p, j);",
     "double dphi[12]; /* tjac^{-1} * dshape : dim x nlb */\n        for (int r = 0; r < dim; r++)\n"
     "            for (int j = 0; j < nlb; j++) {\n                double acc = 0.0;\n"
     "                for (int p = 0; p < dim; p++) acc += AT(tinv, dim, p, r) * AT(ds, dim, p, j);"),
    ("stiffness off-diagonal halved",
     "if (Ke) Ke[e * nlb * nlb + a + b * nlb] = w1 * adet * acc;",
     "if (Ke) Ke[e * nlb * nlb + a + b * nlb] = w1 * adet * acc * (a == b ? 1.0 : 0.5);"),
    ("mass integrand uses phi_a twice",
     "for (int q = 0; q < nq; q++) m += wq[q] * adet * lam[q][a] * lam[q][b];",
     "for (int q = 0; q < nq; q++) m += wq[q] * adet * lam[q][a] * lam[q][a];"),
    ("mass rule point moved",
     "double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0", "double a = (5.0 + 2.0 * sqrt(5.0)) / 20.0"),
    ("centroid rule weight wrong in 3-D",
     "w[0] = (dim == 2) ? 0.5 : 1.0 / 6.0;", "w[0] = (dim == 2) ? 0.5 : 1.0 / 4.0;"),
    ("sparse() keeps the last contribution instead of the sum",
     "if (Ke) { sk += Ke[p];", "if (Ke) { sk = Ke[p];"),
    ("a face of the tetrahedron listed with reversed orientation",
     "{{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}}", "{{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 2, 1}}"),
    ("integration point with the wrong coordinate",
     "x += lam[q * nv + j] * coords[v * dim + i];", "x += lam[q * nv + j] * coords[v * dim + (i + 1) % dim];"),
    ("GI without the rule's weights",
     "for (int q = 0; q < nq; q++) s += w[q] * fip[(c * nq + q) * d + i];",
     "for (int q = 0; q < nq; q++) s += fip[(c * nq + q) * d + i];"),
    ("P2 vertex function wrong",
     "phi[i] = lam[i] * (2.0 * lam[i] - 1.0);", "phi[i] = lam[i] * (2.0 * lam[i] - 0.5);"),
    ("P2 edge gradient loses a term",
     "gphi[r + t * dim] = 4.0 * (lam[i] * glam[r + j * dim] + lam[j] * glam[r + i * dim]);",
     "gphi[r + t * dim] = 4.0 * (lam[i] * glam[r + j * dim]);"),
    ("element integration point with the wrong coordinate",
     "x += lam[q][j] * coords[node * dim + i];", "x += lam[q][j] * coords[node * dim + (i + 1) % dim];"),
    ("stiffness coefficient squared",
     "k += wq[q] * ck * adet * gg;", "k += wq[q] * ck * ck * adet * gg;"),
    ("mass coefficient dropped",
     "m += wq[q] * cm * adet * lam[q][a] * lam[q][b];", "m += wq[q] * adet * lam[q][a] * lam[q][b];"),
    ("det-condition from the second row",
     "s += fabs(AT(a, dim, 0, j) * cof);", "s += fabs(AT(a, dim, 1, j) * cof);"),
    ("edge vectors of coords3D reversed",
     "vectors3d[e * dim * (nlb - 1) + i + j * dim] = coords[node * dim + i] - coords[last * dim + i];",
     "vectors3d[e * dim * (nlb - 1) + i + j * dim] = coords[last * dim + i] - coords[node * dim + i];"),
    ("page scaling by the first page's scalar",
     "c[k * ps + q] = s[k] * a[k * ps + q];", "c[k * ps + q] = s[0] * a[k * ps + q];"),
    ("bilinear form with A transposed",
     "acc += u[k * n + i] * AT(ak, n, i, j) * v[k * n + j];", "acc += u[k * n + i] * AT(ak, n, j, i) * v[k * n + j];"),
    ("determinant scale without absolute values",
     "pabs *= fabs(AT(a, n, i, p[i]));", "pabs *= AT(a, n, i, p[i]);"),
    ("boundary normal: wrong sign of one component (3-D)",
     "n[1] = u[2] * v[0] - u[0] * v[2];", "n[1] = u[0] * v[2] - u[2] * v[0];"),
    ("boundary normal: wrong sign of one component (2-D)",
     "n[1] = coords[ia * 2] - coords[ib * 2];", "n[1] = coords[ib * 2] - coords[ia * 2];"),
    ("load vector with the first basis function only",
     "v += wq[q] * adet * fq[e * nq + q] * lam[q][j];", "v += wq[q] * adet * fq[e * nq + q] * lam[q][0];"),
    ("face's second element repeats the first",
     "fel[nf * 2 + 1] = (j - i == 2) ? (int32_t)all[i + 1].e : -1;",
     "fel[nf * 2 + 1] = (j - i == 2) ? (int32_t)all[i].e : -1;"),
    ("face orientation ignores the element's orientation",
     "FACE3[f->k][det < 0 ? nv - 1 - t : t] : FACE2[f->k][det < 0 ? nv - 1 - t : t]",
     "FACE3[f->k][t] : FACE2[f->k][t]"),
]


def _run_pins(workdir, tag, source):
    c = os.path.join(workdir, f"pf_oracle_{tag}.c")
    with open(c, "w") as f:
        f.write(source)
    so = os.path.join(workdir, f"liboracle_{tag}.so")
    subprocess.run(["gcc", *CFLAGS, "-o", so, c, "-lm"], check=True)
    env = dict(os.environ, PF_ORACLE_LIB=so)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                           PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def test_unchanged_copy_passes_every_pin(tmp_path):
    r = _run_pins(str(tmp_path), "copy", open(SRC).read())
    assert r.returncode == 0, r.stdout[-2000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    """All mutants at once, several pin runs in parallel (each in its own process)."""
    src = open(SRC).read()
    for what, old, _ in MUTATIONS:
        assert src.count(old) == 1, f"the text to mutate is not unique ({what}): {old}"
    jobs = [(i, what, src.replace(old, new)) for i, (what, old, new) in enumerate(MUTATIONS)]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        results = list(pool.map(lambda j: (j[1], _run_pins(str(tmp_path), str(j[0]), j[2])), jobs))
    survivors = [what for what, r in results if r.returncode != 1]
    assert not survivors, f"planted mistakes that passed every pin: {survivors}"
