"""Mutation check of the oracle's pins, run by hand (not collected by pytest):

    python tests/mutation_check.py [substring ...]

(with substrings, only the mutations whose description contains one of them run).

Each mutation plants one plausible mistake in a copy of oracle/pfo.c (a
dropped term, a wrong sign or factor, a wrong index), builds it with the
oracle's own flags, and runs the CPU pins (tests/test_oracle_*.py) against
it through PFO_LIBRARY.  Every mutation must make at least one pin fail; the
script prints which test caught it and exits non-zero if one survives.
Mutations listed in UNPINNED would touch a part with no closed form (stated
as unpinned) and be expected to survive; there are none at present.
"""
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (what the mistake is, [(text in pfo.c, replacement), ...])
MUTATIONS = [
    ("pressure moment without the 1/2 on u.grad rho",
     [("c->pr[q] = s + 0.5 * CS2 * (ux", "c->pr[q] = s + CS2 * (ux")]),
    ("full force instead of half in the momentum moment",
     [("double ux = (jx / CS2 + 0.5 * fx)", "double ux = (jx / CS2 + fx)")]),
    ("receiving-node half of the diffusion term dropped",
     [(" + 0.5 * c->dif[i * n + q] * G;", ";")]),
    ("gravity with the wrong sign in the gbar forcing",
     [("fby = -m.rho * P->g", "fby = m.rho * P->g")]),
    ("shear-rate invariant without the factor 2 on D_xy^2",
     [("2.0 * dxy * dxy", "dxy * dxy")]),
    ("mixed directional derivative with weight 4 instead of 5",
     [("+ 5.0 * at(", "+ 4.0 * at(")]),
    ("surface-tension force with the wrong sign",
     [("sx += c->mu[k * n + q]", "sx -= c->mu[k * n + q]"), ("sy += c->mu[k * n + q]", "sy -= c->mu[k * n + q]")]),
    ("linear mixture viscosity instead of the harmonic one",
     [("if (p->mix_linear) {", "if (!p->mix_linear) {")]),
    ("bounce-back returning the incoming direction",
     [("if (sy < 0 || sy >= c->ny) return c->gpost[(size_t)OPP[a] * n",
       "if (sy < 0 || sy >= c->ny) return c->gpost[(size_t)a * n"),
      ("if (sy < 0 || sy >= c->ny) return c->hpost[((size_t)i * 9 + OPP[a]) * n",
       "if (sy < 0 || sy >= c->ny) return c->hpost[((size_t)i * 9 + a) * n")]),
    ("second-order equilibrium term doubled",
     [("eu * eu / (2.0 * CS2 * CS2)", "eu * eu / (CS2 * CS2)")]),
    ("pressure term of the hbar forcing with the wrong sign",
     [("- cc / (m.rho * CS2) * (ex * bx + ey * by)", "+ cc / (m.rho * CS2) * (ex * bx + ey * by)")]),
    ("gradient term of the chemical potential with the wrong sign",
     [("- 0.75 * p->xi * S[i] * lap[i]", "+ 0.75 * p->xi * S[i] * lap[i]")]),
    ("Laplacian stencil with the centre weight halved",
     [("- 2.0 * c + at(f, x - EX[a]", "- 1.0 * c + at(f, x - EX[a]")]),
    ("central gradient in x with the factor 1/2 dropped",
     [("*gx = sx / (2.0 * CS2);", "*gx = sx / CS2;")]),
    ("power law with exponent n instead of n - 1",
     [("pow(gdot, p->n - 1.0)", "pow(gdot, p->n)")]),
    ("zero shear rate of a shear-thinning liquid taken at nu_min",
     [("if (p->n < 1.0) return p->nu_max;", "if (p->n < 1.0) return p->nu_min;")]),
    ("relaxation time offset by 1/2",
     [("return nu / CS2;", "return nu / CS2 + 0.5;")]),
    ("component densities swapped in the mixture density",
     [("p->rho[0] * clip01(c1) + p->rho[1] * clip01(c2) + p->rho[2] * clip01(c3)",
       "p->rho[2] * clip01(c1) + p->rho[1] * clip01(c2) + p->rho[0] * clip01(c3)")]),
    ("streaming from the downstream neighbour",
     [("int sy = y - EY[a], sx = x - EX[a], n = c->n;", "int sy = y - EY[a], sx = x + EX[a], n = c->n;")]),
    ("hbar relaxation rate 1/tau_h instead of 1/(tau_h + 1/2)",
     [("1.0 / (P->tau_h + 0.5)", "1.0 / P->tau_h")]),
    ("gradient part of the variable-mobility source dropped",
     [("v += c->p.D0 / S[i] * (ax", "v += 0.0 * c->p.D0 / S[i] * (ax")]),
    ("ternary term of the bulk energy with Sigma_1 and Sigma_2 swapped",
     [("c1 * c2 * c3 * (S[0] * c1 + S[1] * c2 + S[2] * c3)", "c1 * c2 * c3 * (S[1] * c1 + S[0] * c2 + S[2] * c3)")]),
    ("six-fold Lambda term of the bulk energy missing a square",
     [("+ p->Lambda * c1 * c1 * c2 * c2 * c3 * c3;", "+ p->Lambda * c1 * c2 * c2 * c3 * c3;")]),
    ("derivative of the bulk energy along C_2 with Sigma_1 in its ternary term",
     [("c1 * c3 * sc + c1 * c2 * c3 * S[1]", "c1 * c3 * sc + c1 * c2 * c3 * S[0]")]),
    ("derivative of the bulk energy along C_1 with half its Lambda term",
     [("+ 2.0 * p->Lambda * c1 * c2 * c2 * c3 * c3;", "+ p->Lambda * c1 * c2 * c2 * c3 * c3;")]),
    ("second component's hbar takes the first component's diffusion source",
     [("double difi = c->dif[i * n + q];", "double difi = c->dif[q];")]),
    ("second component's receiving-node diffusion half from the first component",
     [("+ 0.5 * c->dif[i * n + q] * G;", "+ 0.5 * c->dif[q] * G;")]),
    ("density of component 2 taken from component 1's",
     [("p->rho[1] * clip01(c2)", "p->rho[0] * clip01(c2)")]),
    ("ternary term with Sigma_1 and Sigma_2 swapped in the energy and its derivatives alike",
     [("c1 * c2 * c3 * (S[0] * c1 + S[1] * c2 + S[2] * c3)", "c1 * c2 * c3 * (S[1] * c1 + S[0] * c2 + S[2] * c3)"),
      ("double sc = S[0] * c1 + S[1] * c2 + S[2] * c3;", "double sc = S[1] * c1 + S[0] * c2 + S[2] * c3;"),
      ("+ c2 * c3 * sc + c1 * c2 * c3 * S[0]", "+ c2 * c3 * sc + c1 * c2 * c3 * S[1]"),
      ("+ c1 * c3 * sc + c1 * c2 * c3 * S[1]", "+ c1 * c3 * sc + c1 * c2 * c3 * S[0]")]),
    ("Lambda term read as Lambda C1 C2 C3 in the energy and its derivatives alike",
     [("+ p->Lambda * c1 * c1 * c2 * c2 * c3 * c3;", "+ p->Lambda * c1 * c2 * c3;"),
      ("+ 2.0 * p->Lambda * c1 * c2 * c2 * c3 * c3;", "+ p->Lambda * c2 * c3;"),
      ("+ 2.0 * p->Lambda * c1 * c1 * c2 * c3 * c3;", "+ p->Lambda * c1 * c3;"),
      ("+ 2.0 * p->Lambda * c1 * c1 * c2 * c2 * c3;", "+ p->Lambda * c1 * c2;")]),
    ("outflow without replacing the convected pressure part",
     [("+ W[a] * (pt - (c->pr[q] + U * c->pr[qn]) / (1.0 + U));", ";")]),
    ("outflow pressure extrapolated to the neighbour's value instead of linearly",
     [("double pt = 2.0 * c->pr[qn] - c->pr[qn - 1];", "double pt = c->pr[qn];")]),
    ("inlet y correction with the wrong sign on the diagonal pair",
     [("g[5] += 0.5 * ry;\n            g[8] -= 0.5 * ry;", "g[5] -= 0.5 * ry;\n            g[8] += 0.5 * ry;")]),
    ("inlet unknowns without the odd part of the equilibrium",
     [("if (unknown[a]) g[a] = g[OPP[a]] + gbar_eq(&m, a) - gbar_eq(&m, OPP[a]);", "if (unknown[a]) g[a] = g[OPP[a]];")]),
    ("link-form diffusion source with the node's own mobility at both ends of every link",
     [("s += W[a] * (m0 + m1) * (at(mi,", "s += W[a] * (m0 + m0) * (at(mi,")]),
    ("mass above one half counts cells instead of summing C",
     [("if (cg > 0.5) mh += cg;", "if (cg > 0.5) mh += 1.0;")]),
    ("mean velocity weighted by 1 instead of C",
     [("su += cg * c->u[q];", "su += c->u[q];")]),
    ("centroid height weighted by the clipped C",
     [("sy += cg * y;", "sy += (cg < 0.0 ? 0.0 : (cg > 1.0 ? 1.0 : cg)) * y;")]),
]

# Mistakes in parts that no closed form or invariant reaches (their parity is
# stated as unpinned), expected to survive; none at present.
UNPINNED = []


def build(src_text, tmp):
    with open(os.path.join(tmp, "pfo.c"), "w") as f:
        f.write(src_text)
    shutil.copy(os.path.join(ROOT, "oracle", "pfo.h"), tmp)
    lib = os.path.join(tmp, "libpfo_mutant.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp", "-fPIC",
                    "-shared", os.path.join(tmp, "pfo.c"), "-o", lib, "-lm"], check=True)
    return lib


# pin files in the order they run: the quick ones first, since the run stops
# at the first failing pin
FAST_FIRST = ("thermo", "stencils", "lattice", "diagnostics", "dynamics", "interface", "locality", "mobility",
              "inlet_channel")


def run_pins(lib):
    names = [f for f in os.listdir(os.path.join(ROOT, "tests")) if f.startswith("test_oracle_") and f.endswith(".py")]
    rank = lambda f: next((i for i, k in enumerate(FAST_FIRST) if f == f"test_oracle_{k}.py"), len(FAST_FIRST))
    tests = [os.path.join(ROOT, "tests", f) for f in sorted(names, key=lambda f: (rank(f), f))]
    env = dict(os.environ, PFO_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    failed = [l.split(" ")[1] for l in r.stdout.splitlines() if l.startswith("FAILED ")]
    return r.returncode, failed


def main():
    src = open(os.path.join(ROOT, "oracle", "pfo.c")).read()
    survivors = 0
    only = sys.argv[1:]          # run only the mutations whose description contains one of these
    for what, edits in MUTATIONS + UNPINNED:
        if only and not any(o in what for o in only):
            continue
        pinned = (what, edits) in MUTATIONS
        text = src
        for old, new in edits:
            if old not in text:
                raise SystemExit(f"mutation site not found: {old!r}")
            text = text.replace(old, new)
        with tempfile.TemporaryDirectory() as tmp:
            rc, failed = run_pins(build(text, tmp))
        caught = rc != 0
        survivors += pinned and not caught
        tag = "caught  " if caught else ("SURVIVED" if pinned else "unpinned")
        print(f"{tag}  {what}: {failed[0] if failed else '-'}", flush=True)
    sys.exit(1 if survivors else 0)


if __name__ == "__main__":
    main()
