"""Planted-mistake check of the oracle's pins (run by hand, not collected by
pytest: it takes a few minutes).

Each entry is one plausible single-line mistake in the oracle (a dropped
factor, a wrong sign or index, a transposed operand, a swapped branch).  For
each, the repository is copied to a temporary folder, the mistake is planted
in the copy's oracle, and the CPU test suite (``-m "not gpu"``) must fail.

    python tests/oracle_mutations.py [workers]
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# what the CPU suite needs
COPY = ["oracle", "synth", "tests", "paper_2404_08952_amd", "include", "profiles", "pytest.ini", "bench.py",
        "__graft_entry__.py"]

MUTATIONS = [
    ('oracle/scheme.py',
     '(1.0 - gb) * t[(n, m)]',
     '(1.0 + gb) * t[(n, m)]'),
    ('oracle/scheme.py',
     '(1.0 - 1.0 / gb) * t[(n, m)]',
     '(1.0 - gb) * t[(n, m)]'),
    ('oracle/scheme.py',
     'gb ** (n - 1) * t[(n, m + 1)]',
     'gb ** n * t[(n, m + 1)]'),
    ('oracle/scheme.py',
     'phif = w * phi[P] + (1.0 - w) * phi[N]',
     'phif = (1.0 - w) * phi[P] + w * phi[N]'),
    ('oracle/scheme.py',
     'out.append(2.0 * np.einsum',
     'out.append(1.0 * np.einsum'),
    ('oracle/scheme.py',
     'out.append(4.0 * np.einsum',
     'out.append(2.0 * np.einsum'),
    ('oracle/scheme.py',
     'prod = prod * (xface - xb[..., q])',
     'prod = prod * (xface - xb[..., l])'),
    ('oracle/scheme.py',
     'return np.stack([g ** j for j in range(-r, k - r)], -1)',
     'return np.stack([g ** (-j) for j in range(-r, k - r)], -1)'),
    ('oracle/geometry.py',
     'omega = dN / (dP + dN)',
     'omega = dP / (dP + dN)'),
    ('oracle/flux.py',
     'return np.where((an >= 0.0)[:, None], an[:, None] * UL, an[:, None] * UR)',
     'return np.where((an >= 0.0)[:, None], an[:, None] * UR, an[:, None] * UL)'),
    ('oracle/flux.py',
     'return 0.5 * (FL + FR) - 0.5 * (lam * area)[:, None] * (UR - UL)',
     'return 0.5 * (FL + FR) + 0.5 * (lam * area)[:, None] * (UR - UL)'),
    ('oracle/flux.py',
     'Us[:, 1 + D] = fac * (E / r + (Ss - q) * (Ss + p / (r * (Sk - q))))',
     'Us[:, 1 + D] = fac * (E / r + (Ss - q) * (Ss - p / (r * (Sk - q))))'),
    ('oracle/solver.py',
     'return U / 3.0 + (2.0 / 3.0) * (U2 + dt * rhs(U2))',
     'return U / 3.0 + (2.0 / 3.0) * (U1 + dt * rhs(U2))'),
    ('oracle/geometry.py',
     'cen = (e + fc + q1 + q2) / 4.0',
     'cen = (e + fc + q1 + q2) / 3.0'),
    ('oracle/indicator.py',
     'g0 = 2.0 * np.einsum("fa,fa->f", gq[c, k], d0)',
     'g0 = 1.0 * np.einsum("fa,fa->f", gq[c, k], d0)'),
    ('oracle/indicator.py',
     'beta = np.abs(s - delta) / (np.abs(s) + np.abs(delta) + eps)',
     'beta = np.abs(s + delta) / (np.abs(s) + np.abs(delta) + eps)'),
    ('oracle/indicator.py',
     'r = np.clip(s * delta / (delta * delta + eps * eps), -2.0, 2.0)',
     'r = np.clip(s * delta / (delta * delta + eps * eps), -1.0, 2.0)'),
    ('oracle/indicator.py',
     'scale = np.abs(q[:, k]) + sum_dl / cnt + 1e-8',
     'scale = np.abs(q[:, k]) + sum_dl + 1e-8'),
    ('oracle/indicator.py',
     'Z2 = r(H1) @ r(W2).T + b2',
     'Z2 = r(H1) @ r(W2) + b2'),
    ('oracle/indicator.py',
     'd1 = (d2b @ r(W2)) * (1 - H1 * H1)',
     'd1 = (d2b @ r(W2)) * (1 - H1)'),
    ('oracle/indicator.py',
     'g3 = (th - y) / n',
     'g3 = (y - th) / n'),
    ('oracle/indicator.py',
     'return params - lr * mh / (np.sqrt(vh) + eps), m, v',
     'return params + lr * mh / (np.sqrt(vh) + eps), m, v'),
    ('oracle/limiter.py',
     'return np.where(prod > 0.0, 2.0 * prod / safe, 0.0)',
     'return np.where(prod > 0.0, 1.0 * prod / safe, 0.0)'),
    ('oracle/boundary.py',
     'UO = UC + 2.0 * (Tf - UC)',
     'UO = UC + 1.0 * (Tf - UC)'),
    ('oracle/boundary.py',
     'Tf = np.where((typ == NEUMANN)[:, None], UC + val * X.dist[:, None], Tf)',
     'Tf = np.where((typ == NEUMANN)[:, None], UC - val * X.dist[:, None], Tf)'),
    ('oracle/boundary.py',
     'GO = np.where((typ == DIRICHLET)[:, None, None], -GO, GO)',
     'GO = np.where((typ == DIRICHLET)[:, None, None], GO, GO)'),
    ('oracle/scheme.py',
     'alpha = [dl[:, k].reshape(shape) / (WENO_EPS + beta[k]) ** 2 for k in range(3)]',
     'alpha = [dl[:, k].reshape(shape) / (WENO_EPS + beta[k]) ** 1 for k in range(3)]'),
    ('oracle/scheme.py',
     '(4.0 / 3.0) * a[:, 2] ** 2 + 4.0 * a[:, 2] ** 2)',
     '(4.0 / 3.0) * a[:, 2] ** 2 + 0.0 * a[:, 2] ** 2)'),
    ('oracle/scheme.py',
     'r_if_left = np.where(np.abs(d3_m2) < keep * np.abs(d3_m1), 2, 1)',
     'r_if_left = np.where(np.abs(d3_m2) < keep * np.abs(d3_m1), 1, 2)'),
    ('oracle/scheme.py',
     'UR = side(GN, GP, -geo.d, 1.0 / geo.g, scheme)',
     'UR = side(GN, GP, -geo.d, geo.g, scheme)'),
    ('oracle/scheme.py',
     'UR = side(GN, GP, -geo.d, 1.0 / geo.g, scheme)',
     'UR = side(GN, GP, geo.d, 1.0 / geo.g, scheme)'),
    # blend, sensor, positivity and indicator channels
    ('oracle/limiter.py',
     'return np.clip((BETA_HI - beta) / (BETA_HI - BETA_LO), 0.0, 1.0), beta',
     'return np.clip((BETA_HI - beta) / (BETA_HI + BETA_LO), 0.0, 1.0), beta'),
    ('oracle/limiter.py',
     'np.maximum.at(beta, N, bN)',
     'np.maximum.at(beta, P, bN)'),
    ('oracle/limiter.py',
     'tf = np.minimum(theta[mesh.owner], theta[mesh.neighbour])[:, None]',
     'tf = np.maximum(theta[mesh.owner], theta[mesh.neighbour])[:, None]'),
    ('oracle/limiter.py',
     'UR = U[N] + limited_increment(sR, dR, w)',
     'UR = U[N] + limited_increment(sR, dR, 1.0 - w)'),
    ('oracle/limiter.py',
     'return np.where(np.abs(inc) > np.abs(delta), delta, inc)',
     'return inc'),
    ('oracle/solver.py',
     'UR = np.where(badR[:, None], U[mesh.neighbour], UR)',
     'UR = np.where(badR[:, None], U[mesh.owner], UR)'),
    ('oracle/indicator.py',
     'g_p = (gamma - 1.0) * (g_E - u_dot_gm',
     'g_p = (gamma - 1.0) * (g_E + u_dot_gm'),
    ('oracle/indicator.py',
     'np.einsum("ca,cad->cd", m / safe[:, None], g_m)',
     'np.einsum("ca,cda->cd", m / safe[:, None], g_m)'),
    ('oracle/indicator.py',
     'f = np.stack([acc_max[0] / scale,',
     'f = np.stack([acc_max[0] / scale ** 2,'),
    ('oracle/indicator.py',
     'acc_max[2], sum_beta / cnt, acc_min,',
     'acc_max[2], sum_beta, acc_min,'),
    ('oracle/indicator.py',
     'acc_max[3] / scale], 1)',
     'acc_max[3]], 1)'),
]


def check(item):
    i, (path, old, new) = item
    tmp = tempfile.mkdtemp(prefix=f"oracle_mut{i}_")
    try:
        dst = os.path.join(tmp, "repo")
        os.makedirs(dst)
        skip = shutil.ignore_patterns("__pycache__", "*.so", "*.o")
        for name in COPY:
            src_path = os.path.join(ROOT, name)
            if os.path.isdir(src_path):
                shutil.copytree(src_path, os.path.join(dst, name), ignore=skip)
            else:
                shutil.copy2(src_path, os.path.join(dst, name))
        p = os.path.join(dst, path)
        with open(p) as fh:
            src = fh.read()
        if old not in src:
            return f"NOT FOUND  {path}: {old[:60]}"
        with open(p, "w") as fh:
            fh.write(src.replace(old, new, 1))
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                            "--ignore=tests/test_host_abi.py", "tests"], cwd=dst, capture_output=True, text=True,
                           env=dict(os.environ, OMP_NUM_THREADS="1"))
        failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")][:1]
        verdict = "caught" if r.returncode != 0 else "MISSED"
        return f"{verdict:10s} {path}: {old[:60]}  {failed[0][7:80] if failed else ''}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    # control: the copy without a planted mistake must pass
    path, old, _new = MUTATIONS[0]
    control = check((len(MUTATIONS), (path, old, old)))
    print("control (no mistake):", "passes" if control.startswith("MISSED") else "FAILS", flush=True)
    if not control.startswith("MISSED"):
        sys.exit(2)
    missed = 0
    with cf.ThreadPoolExecutor(workers) as ex:
        for line in ex.map(check, enumerate(MUTATIONS)):
            print(line, flush=True)
            missed += not line.startswith("caught")
    print(f"{len(MUTATIONS) - missed} of {len(MUTATIONS)} planted mistakes caught")
    sys.exit(1 if missed else 0)


if __name__ == "__main__":
    main()
