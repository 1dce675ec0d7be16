"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped factor, a wrong sign or index, a
transposed operand) in a copy of the oracle's C source, builds it on the CPU
and runs the pin suite against it in a subprocess: the suite has to fail.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bd3mg_oracle.c")
NET_SRC = os.path.join(ROOT, "oracle", "convnet_oracle.c")

MUTATIONS = {
    "box-gradient-factor": ("acc += 2.0 * p->eta * (x[v]", "acc += 1.0 * p->eta * (x[v]"),
    "box-curvature-factor": ("return quad + 2.0 * p->eta * box", "return quad + 1.0 * p->eta * box"),
    "tv-adjoint-sign": ("if (i >= 1) tv += omega_at(p, x, k, j, i - 1) * dX(p, x, k, j, i - 1);",
                        "if (i >= 1) tv -= omega_at(p, x, k, j, i - 1) * dX(p, x, k, j, i - 1);"),
    "tv-adjoint-weight-index": ("if (j >= 1) tv += omega_at(p, x, k, j - 1, i) * dY(p, x, k, j - 1, i);",
                                "if (j >= 1) tv += omega_at(p, x, k, j, i) * dY(p, x, k, j - 1, i);"),
    "tv-curvature-drops-y": ("double d = dX(p, u, k, j, i) * dX(p, v, k, j, i) + dY(p, u, k, j, i) * dY(p, v, k, j, i);",
                             "double d = dX(p, u, k, j, i) * dX(p, v, k, j, i);"),
    "omega-delta-not-squared": ("return 1.0 / sqrt(gxv * gxv + gyv * gyv + gzv * gzv + p->delta * p->delta);",
                                "return 1.0 / sqrt(gxv * gxv + gyv * gyv + gzv * gzv + p->delta);"),
    "blur-transposed": ("int sg = transpose ? 1 : -1;", "int sg = transpose ? -1 : 1;"),
    "adjoint-z-weight-of-output-slice": ("acc += p->gz[(size_t)m * p->kz + (c + rz)]",
                                         "acc += p->gz[(size_t)k * p->kz + (c + rz)]"),
    "step-sign": ("double u2 = -(P[1] * c1 + P[2] * c2);", "double u2 = (P[1] * c1 + P[2] * c2);"),
    "pinv-offdiagonal-sign": ("P[1] = -b12 / det;", "P[1] = b12 / det;"),
    "coloring-gap-off-by-one": ("if (gap < min_gap) { ok = 0; break; }",
                                "if (gap < min_gap - 1) { ok = 0; break; }"),
    "z-penalty-factor": ("zz -= dZ(p, x, k, j, i);\n                    acc += 2.0 * p->kappa * zz;",
                         "zz -= dZ(p, x, k, j, i);\n                    acc += p->kappa * zz;"),
    "inflation-dropped": ("B[0] += p->mu * dot_slices(p, d1, d1, z0, z0 + n);",
                          "B[0] += 0.0 * dot_slices(p, d1, d1, z0, z0 + n);"),
    "round-applies-in-sequence": ("            block_direction(p, x, dprev, z0, nslices[b], dn, NULL);\n",
                                  "            block_direction(p, x, dprev, z0, nslices[b], dn, NULL);\n"
                                  "            for (size_t q = (size_t)z0 * nslice(p); q < (size_t)(z0 + nslices[b]) * nslice(p); ++q)"
                                  " { x[q] += dn[q]; dprev[q] = dn[q]; dn[q] = 0.0; }\n"),
    "lipschitz-tv-term": ("return hh + 2.0 * p->eta + tvc * p->lambda / p->delta",
                          "return hh + 2.0 * p->eta + p->lambda / p->delta"),
    "dense-kernel-of-input-slice": ("double w = psf_w(p, k, c, b, a);", "double w = psf_w(p, kk, c, b, a);"),
    "dense-adjoint-kernel-of-output-slice": ("double w = psf_w(p, kk, c, b, a);", "double w = psf_w(p, k, c, b, a);"),
    "dense-tap-flipped-in-z": ("p->pk[(((size_t)k * p->kz + (c + rz)) * p->ky",
                               "p->pk[(((size_t)k * p->kz + (rz - c)) * p->ky"),
    "rotation-direction": ("double u = a * ct + b * st, v = -a * st + b * ct;",
                           "double u = a * ct - b * st, v = a * st + b * ct;"),
    "majorant-apply-box-factor": ("double acc = out[v] + 2.0 * p->eta * u[v];",
                                  "double acc = out[v] + 1.0 * p->eta * u[v];"),
    "majorant-apply-tv-weight-index": ("if (i >= 1) tv += omega_at(p, x, k, j, i - 1) * dX(p, u, k, j, i - 1);",
                                       "if (i >= 1) tv += omega_at(p, x, k, j, i) * dX(p, u, k, j, i - 1);"),
    "bicg-residual-sign": ("r[q] -= alpha * ap[q];", "r[q] += alpha * ap[q];"),
    "bicg-direction-update": ("pv[q] = r[q] + beta * pv[q];", "pv[q] = r[q] + rho * pv[q];"),
    "async-gd-step-without-L": ("u1 = B[0] > 0.0 ? -c1 / B[0] : 0.0;", "u1 = B[0] > 0.0 ? -c1 / gg : 0.0;"),
    "async-cg-metric-offdiagonal-sign": ("B[1] = -lm * gd;", "B[1] = lm * gd;"),
    "dense-lipschitz-column-sums": ("if (k + t >= 0 && k + t < p->nz) c += fabs(p->pk[((size_t)(k + t) * p->kz + t + rz) * kk + q]);",
                                    "if (k + t >= 0 && k + t < p->nz) c += 0.5 * fabs(p->pk[((size_t)(k + t) * p->kz + t + rz) * kk + q]);"),
    "tv3d-omega-drops-z": ("double gzv = p->tv3d ? dZ(p, x, k, j, i) : 0.0;", "double gzv = 0.0;"),
    "tv3d-f-drops-z": ("double g3 = p->tv3d ? gzv : 0.0;", "double g3 = 0.0;"),
    "tv3d-adjoint-z-sign": ("if (k >= 1) tv += omega_at(p, x, k - 1, j, i) * dZ(p, x, k - 1, j, i);",
                            "if (k >= 1) tv -= omega_at(p, x, k - 1, j, i) * dZ(p, x, k - 1, j, i);"),
    "tv3d-form-misses-the-slice-below": ("int t0 = (p->tv3d && z0 >= 1) ? z0 - 1 : z0;", "int t0 = z0;"),
    "tv3d-lipschitz-keeps-8": ("double tvc = p->tv3d ? 12.0 : 8.0;", "double tvc = 8.0;"),
}

NET_MUTATIONS = {
    "net-skip-concat-dropped": ("memcpy(A->cat1 + c * V1, A->s1, c * V1 * sizeof(double));",
                                "memset(A->cat1 + c * V1, 0, c * V1 * sizeof(double));"),
    "net-pool-divisor": ("out[(((size_t)c * d + z) * h + y) * w + x] = s / 8.0;",
                         "out[(((size_t)c * d + z) * h + y) * w + x] = s / 4.0;"),
    "net-conv-tap-flipped": ("const int zz = z + a - r, yy = y + bb - r, xx = x + cc - r;\n"
                             "                                    if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;\n"
                             "                                    const double wv",
                             "const int zz = z - a + r, yy = y + bb - r, xx = x + cc - r;\n"
                             "                                    if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;\n"
                             "                                    const double wv"),
    "net-relu-mask-on-wrong-tensor": ("relu_bwd(A.c1, gc1, c * V1);", "relu_bwd(A.e1, gc1, c * V1);"),
    "net-skip-gradient-dropped": ("for (size_t i = 0; i < 2 * c * V2; ++i) gs2[i] += gcat2[2 * c * V2 + i];",
                                  "(void)gcat2;"),
    "net-bf16-ties-away": ("u += 0x7fffu + lsb;", "u += 0x8000u; (void)lsb;"),
}

PIN_FILES = {SRC: ["test_oracle_pins.py", "test_oracle_round.py", "test_oracle_dense.py",
                   "test_oracle_ablation.py", "test_oracle_tv3d.py"],
             NET_SRC: ["test_oracle_convnet.py"]}


def _cases():
    return [(SRC, n, MUTATIONS[n]) for n in sorted(MUTATIONS)] + \
           [(NET_SRC, n, NET_MUTATIONS[n]) for n in sorted(NET_MUTATIONS)]


def _run_case(path, name, edit, work):
    """Build the oracle with one planted mistake and run its pins; returns
    (pins' exit status, the tail of their output), or None when the pattern
    does not occur exactly once."""
    old, new = edit
    src = open(path).read()
    if src.count(old) != 1:
        return None
    d = os.path.join(work, name)
    os.makedirs(d)
    mut = os.path.join(d, "mut.c")
    with open(mut, "w") as fh:
        fh.write(src.replace(old, new))
    others = [s for s in PIN_FILES if s != path]
    lib = os.path.join(d, "libmut.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-o", lib, mut] + others + ["-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] +
                         [os.path.join(ROOT, "tests", f) for f in PIN_FILES[path]],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return res.returncode, res.stdout[-2000:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Every case at once, a few processes at a time (the pins of one case
    run single-threaded), so the module takes minutes rather than the sum."""
    work = str(tmp_path_factory.mktemp("mutations"))
    workers = max(1, min(6, (os.cpu_count() or 2) - 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {c[1]: ex.submit(_run_case, c[0], c[1], c[2], work) for c in _cases()}
        return {n: f.result() for n, f in futs.items()}


@pytest.mark.parametrize("path,name,edit", _cases(), ids=[c[1] for c in _cases()])
def test_pins_catch_planted_mistake(path, name, edit, outcomes):
    out = outcomes[name]
    assert out is not None, "pattern of %s does not occur exactly once" % name
    rc, tail = out
    assert rc != 0, "pins did not catch mutation %s\n%s" % (name, tail)
