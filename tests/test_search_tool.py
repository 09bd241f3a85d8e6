"""The flip-graph search tool (paper_1409_2908_amd/algorithms/search.py and
search.c): the schemes it writes pass the oracle's exact Brent check, and
every shipped table it produced names the command that regenerates it.
CPU only (gcc builds the walker)."""
import os
import re
import subprocess
import sys

import pytest

from oracle import tensor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ALGS = os.path.join(ROOT, "paper_1409_2908_amd", "algorithms")
SEARCH = os.path.join(ALGS, "search.py")


def _parse(text):
    rows = [[int(t) for t in l.split()] for l in text.splitlines() if l.strip() and not l.startswith("#")]
    M, K, N, R = rows[0]
    body = rows[1:]
    assert len(body) == M * K + K * N + M * N
    return M, K, N, R, body[:M * K], body[M * K:M * K + K * N], body[M * K + K * N:]


@pytest.mark.parametrize("over", ["z", "gf2"])
def test_search_writes_brent_exact_strassen_rank(over, tmp_path):
    out = tmp_path / "t.txt"
    subprocess.run([sys.executable, SEARCH, "2", "2", "2", "7", "--seeds", "1-2", "--count", "2",
                    "--plateau", "1000", "--over", over, "--out", str(out)], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=300)
    text = out.read_text()
    assert "Regenerate: python paper_1409_2908_amd/algorithms/search.py 2 2 2 7 --seeds 1-2" in text
    M, K, N, R, U, V, W = _parse(text)
    assert (M, K, N, R) == (2, 2, 2, 7)
    assert all(x in (-1, 0, 1) for row in U + V + W for x in row)
    assert tensor.brent_residual(U, V, W, M, K, N) == []


@pytest.mark.parametrize("dims", [("2", "2", "2", "7"), ("3", "2", "2", "11")])
def test_search_2adic_lift_is_brent_exact(dims, tmp_path):
    """GF(2) walks with the 2-adic lift enabled: whatever lift is taken, the
    written scheme passes the oracle's own exact Brent check and names the
    lift in its regeneration command."""
    out = tmp_path / "t.txt"
    subprocess.run([sys.executable, SEARCH, *dims, "--seeds", "1-2", "--count", "2", "--plateau", "2000",
                    "--over", "gf2", "--lift", "2adic", "--out", str(out)], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=300)
    text = out.read_text()
    assert "--over gf2 --lift 2adic" in text
    M, K, N, R, U, V, W = _parse(text)
    assert (M, K, N, R) == tuple(int(d) for d in dims)
    assert tensor.brent_residual(U, V, W, M, K, N) == []


def test_2adic_lift_of_strassen_mod_2():
    """Strassen's scheme reduced modulo 2 lifts back to an exact integer
    scheme (the Hensel steps reach a solution over the integers)."""
    sys.path.insert(0, ALGS)
    import search
    from oracle import algorithms
    a = algorithms.get("strassen_222_7")
    scheme = []
    for r in range(a.R):
        masks = [sum(((X[i][r] & 1) << i) for i in range(len(X))) for X in (a.U, a.V, a.W)]
        scheme.append(tuple(masks))
    lifted = search.lift_2adic(2, 2, 2, scheme)
    assert lifted is not None
    U, V, W = lifted
    assert tensor.brent_residual(U, V, W, 2, 2, 2) == []
    # same support as the GF(2) scheme, entries +-1 there
    for X, Y in ((U, a.U), (V, a.V), (W, a.W)):
        for row, ref in zip(X, Y):
            assert [abs(x) for x in row] == [abs(y) for y in ref]


def test_search_is_deterministic_per_seed(tmp_path):
    outs = []
    for i in range(2):
        out = tmp_path / f"t{i}.txt"
        subprocess.run([sys.executable, SEARCH, "3", "2", "2", "11", "--seeds", "3", "--count", "1",
                        "--plateau", "2000", "--out", str(out)], check=True,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=300)
        outs.append(out.read_text())
    assert outs[0] == outs[1]
    M, K, N, R, U, V, W = _parse(outs[0])
    assert R == 11 and tensor.brent_residual(U, V, W, M, K, N) == []


@pytest.mark.parametrize("name", ["fmm_323_15", "fmm_423_20", "fmm_424_26", "fmm_334_29", "fmm_434_38"])
def test_shipped_searched_tables_name_their_command(name):
    text = open(os.path.join(ALGS, name + ".txt")).read()
    m = re.search(r"Regenerate: python paper_1409_2908_amd/algorithms/search.py (\d) (\d) (\d) (\d+) ", text)
    assert m, name
    M, K, N, R, U, V, W = _parse(text)
    assert tuple(int(x) for x in m.groups()) == (M, K, N, R)
    assert tensor.brent_residual(U, V, W, M, K, N) == []
    nz = sum(1 for row in U + V + W for x in row if x)
    assert f"{nz} non-zeros" in text
