"""The oracle's pins catch plausible mistakes in the oracle.

Each entry below plants one mistake in a copy of ``oracle/clbm_oracle.c`` (a dropped term,
a wrong sign, factor or index, a transposed operand, a mistyped matrix entry), builds the
copy with the oracle's own build flags, and runs the oracle pin tests against it (the
files named in PINS, through ``CLBM_ORACLE_LIB``). Every mutant must make at least one pin
fail. Each original snippet must occur exactly once in the source, so a change of the
oracle that moves a snippet fails this test instead of silently skipping a mutant.
Runs on the CPU only; the mistakes are planted in the oracle, never in the GPU library.
"""
import concurrent.futures
import os
import re
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = ["tests/test_oracle_matrices.py", "tests/test_oracle_collision.py",
        "tests/test_oracle_relaxation.py", "tests/test_oracle_analytic.py",
        "tests/test_oracle_viscous.py", "tests/test_oracle_source_field.py"]

# (what the mistake is, original snippet, mutated snippet)
MUTANTS = [
    ("Eq. (6a): one sign of the k21 row",
     "    {0, 0, 0, 0, 0, 1, 1, -1, -1},\n", "    {0, 0, 0, 0, 0, 1, -1, -1, -1},\n"),
    ("Eq. (16): one entry of the k02 row",
     "    {0, 0, 1, 0, 1},\n};", "    {0, 0, 1, 1, 1},\n};"),
    ("Eq. (6b): factor 2 dropped in the k20 shift",
     "N[3][0] = ux2;            N[3][1] = -2 * ux;", "N[3][0] = ux2;            N[3][1] = -ux;"),
    ("Eq. (6b): k21 shift takes +u_y k20",
     "N[6][3] = -uy;", "N[6][3] = uy;"),
    ("Eq. (6b): factor 4 of k11 in the k22 shift halved",
     "N[8][5] = 4 * ux * uy;", "N[8][5] = 2 * ux * uy;"),
    ("Eq. (6b): k12 and k21 shifts of k22 transposed",
     "N[8][6] = -2 * uy;        N[8][7] = -2 * ux;", "N[8][6] = -2 * ux;        N[8][7] = -2 * uy;"),
    ("Eq. (17): u_x^2 term of the thermal k20 shift dropped",
     "N[3][0] = ux * ux;", "N[3][0] = 0.0;"),
    ("Sec. 3: no-slip rule for s_3 with a wrong sign",
     "(16.0 - 8.0 * s_nu) / (8.0 - s_nu)", "(16.0 - 8.0 * s_nu) / (8.0 + s_nu)"),
    ("Sec. 3.1: lambda_2 rule with a wrong sign",
     "12.0 * (l1 - 2.0) / (l1 - 12.0)", "12.0 * (l1 - 2.0) / (l1 + 12.0)"),
    ("Sec. 2.2: lambda_1 from c_s^2 instead of c_T^2",
     "1.0 / (p->alpha / CT2 + 0.5)", "1.0 / (p->alpha / CS2 + 0.5)"),
    ("Eq. (8): bulk and shear parts of the 2nd-order block swapped",
     "c->S[3 * Q9 + 3] = sp; c->S[3 * Q9 + 4] = sm;", "c->S[3 * Q9 + 3] = sm; c->S[3 * Q9 + 4] = sp;"),
    ("Eq. (8): s_3 in place of s_4 on k22",
     "c->S[8 * Q9 + 8] = c->s_4;", "c->S[8 * Q9 + 8] = c->s_3;"),
    ("Eq. (8): a caller's s_4 ignored (always 1)",
     "double s_4 = isnan(p->s_4) ? 1.0 : p->s_4;", "double s_4 = 1.0;"),
    ("Eq. (8): a caller's s_b ignored (always 1)",
     "double s_b = isnan(p->s_b) ? 1.0 : p->s_b;", "double s_b = 1.0;"),
    ("Eq. (8): bulk rate ignored, the trace relaxed at s_nu",
     "double sp = 0.5 * (c->s_b + c->s_nu), sm = 0.5 * (c->s_b - c->s_nu);",
     "double sp = c->s_nu, sm = 0.0;"),
    ("Eq. (8): s- with the wrong sign",
     "double sp = 0.5 * (c->s_b + c->s_nu), sm = 0.5 * (c->s_b - c->s_nu);",
     "double sp = 0.5 * (c->s_b + c->s_nu), sm = 0.5 * (c->s_nu - c->s_b);"),
    ("Eq. (8): the collision uses s_4 = 1 whatever the rates say",
     "c->s_3 = r[2]; c->s_4 = r[3];", "c->s_3 = r[2]; c->s_4 = 1.0;"),
    ("S_T: lambda_2 on the first thermal moments",
     "c->ST[1 * Q5 + 1] = c->l1; c->ST[2 * Q5 + 2] = c->l1;",
     "c->ST[1 * Q5 + 1] = c->l2; c->ST[2 * Q5 + 2] = c->l2;"),
    ("S_T: lambda_1 on the second thermal moments",
     "c->ST[3 * Q5 + 3] = c->l2; c->ST[4 * Q5 + 4] = c->l2;",
     "c->ST[3 * Q5 + 3] = c->l1; c->ST[4 * Q5 + 4] = c->l1;"),
    ("Eq. (25): source correction of T with a wrong sign",
     "    T += 0.5 * Qn;", "    T -= 0.5 * Qn;"),
    ("Eq. (2): buoyancy with a wrong sign",
     "double Fy = p->Fy + p->g_beta * (T - p->T0);", "double Fy = p->Fy - p->g_beta * (T - p->T0);"),
    ("Eq. (12): the whole force in the velocity",
     "    double ux = (jx + 0.5 * Fx) / rho;", "    double ux = (jx + Fx) / rho;"),
    ("Eq. (7): force term without the 1/2 of (I - S/2)",
     "(I - 0.5 * Srk) * C[k];", "(I - Srk) * C[k];"),
    ("Eq. (10): third-order force terms transposed",
     "CS2 * Fy, CS2 * Fx, 0};", "CS2 * Fx, CS2 * Fy, 0};"),
    ("Eq. (9): k22 equilibrium rho c_s^2 in the collision",
     "rho * CS2 * CS2};\n    double C[Q9]", "rho * CS2};\n    double C[Q9]"),
    ("Eq. (24): second-order source terms dropped",
     "double R[Q5] = {Qn, 0, 0, Qn * CT2, Qn * CT2};", "double R[Q5] = {Qn, 0, 0, 0, 0};"),
    ("Eq. (23): source term without the 1/2 of (I - S/2)",
     "(I - 0.5 * Srk) * R[k];", "(I - Srk) * R[k];"),
    ("Eq. (19): thermal equilibrium with c_s^2 in the collision",
     "double kteq[Q5] = {T, 0, 0, T * CT2, T * CT2};\n    double R", "double kteq[Q5] = {T, 0, 0, T * CS2, T * CS2};\n    double R"),
    ("Eq. (9): k22 equilibrium rho c_s^2 at initialisation",
     "rho * CS2 * CS2};\n    double kteq", "rho * CS2};\n    double kteq"),
    ("Eq. (11): populations streamed against their velocity",
     "crossed_sides(p, x, y, EX[i], EY[i], &tx, &ty, &xs, &ys);", "crossed_sides(p, x, y, -EX[i], -EY[i], &tx, &ty, &xs, &ys);"),
    ("Sec. 3: bounce-back into the same population",
     "s->fn[k * Q9 + ib] = s->fp[k * Q9 + i] - 2.0", "s->fn[k * Q9 + i] = s->fp[k * Q9 + i] - 2.0"),
    ("moving wall: momentum term with a wrong sign",
     "s->fp[k * Q9 + i] - 2.0 * s->w[i]", "s->fp[k * Q9 + i] + 2.0 * s->w[i]"),
    ("Eq. (26): c_T^2 dropped from the anti-bounce-back",
     "-s->gp[k * Q5 + i] + CT2 * Tw;", "-s->gp[k * Q5 + i] + Tw;"),
    ("Eq. (26): bounce-back instead of anti-bounce-back",
     "-s->gp[k * Q5 + i] + CT2 * Tw;", "s->gp[k * Q5 + i];"),
    ("Eq. (28): second-layer temperature with a wrong sign",
     "(9.0 * b1 * T1 - b1 * T2 + 3.0 * ne * dx * b3)", "(9.0 * b1 * T1 + b1 * T2 + 3.0 * ne * dx * b3)"),
    ("Eq. (28): factor 3 of b2 dropped",
     "(8.0 * b1 + 3.0 * ne * dx * b2)", "(8.0 * b1 + ne * dx * b2)"),
    ("Eq. (27): T2 taken at the wall node itself",
     "double T2 = s->T[(size_t)y2 * nx + x2];", "double T2 = s->T[k];"),
    ("Sec. 3.2: factor 2 of the normal strain dropped",
     "(cen[3] - cen[4]) / (2.0 * CS2 * rho);", "(cen[3] - cen[4]) / (CS2 * rho);"),
    ("source field ignored",
     "((p->Q_field && k >= 0) ? p->Q_field[k] : 0.0)", "0.0"),
    ("source field read at the previous node",
     "((p->Q_field && k >= 0) ? p->Q_field[k] : 0.0)", "((p->Q_field && k >= 0) ? p->Q_field[k > 0 ? k - 1 : k] : 0.0)"),
    ("source field counted twice",
     "((p->Q_field && k >= 0) ? p->Q_field[k] : 0.0)", "((p->Q_field && k >= 0) ? 2.0 * p->Q_field[k] : 0.0)"),
    ("Sec. 3.2: shear strain rate halved",
     "double shear = -c->s_nu * cen[5] / (CS2 * rho);", "double shear = -c->s_nu * cen[5] / (CS2 * rho) * 0.5;"),
]


def _run_mutant(idx, src, tmp):
    what, orig, mut = MUTANTS[idx]
    d = os.path.join(tmp, "m%02d" % idx)
    os.makedirs(d)
    with open(os.path.join(d, "clbm_oracle.c"), "w") as fh:
        fh.write(src.replace(orig, mut))
    shutil.copy(os.path.join(ORACLE, "clbm_oracle.h"), d)
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    lib = oracle_build.build(src_dir=d, out=os.path.join(d, "liboracle.so"))
    env = dict(os.environ, CLBM_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"] + PINS,
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=600)
    caught = re.findall(r"^FAILED (\S+)", r.stdout, re.M)
    return idx, r.returncode, caught[0] if caught else ""


def test_every_mutant_fails_a_pin():
    with open(os.path.join(ORACLE, "clbm_oracle.c")) as fh:
        src = fh.read()
    for what, orig, mut in MUTANTS:
        assert src.count(orig) == 1, "snippet for '%s' not found exactly once" % what
        assert orig != mut
    tmp = tempfile.mkdtemp(prefix="oracle_mutants_")
    try:
        with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
            results = sorted(ex.map(lambda i: _run_mutant(i, src, tmp), range(len(MUTANTS))))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    survivors = []
    for idx, rc, caught in results:
        print("%-62s rc %d  %s" % (MUTANTS[idx][0], rc, caught or "(no pin failed)"), flush=True)
        if rc != 1 or not caught:
            survivors.append(MUTANTS[idx][0])
    assert not survivors, "mutants no pin caught: %s" % survivors
