"""Search for bilinear base cases <M,K,N;R> with integer coefficients.

Section 2.3 of the paper finds fast algorithms numerically (alternating least
squares with regularisation, then rounding); this tool takes the discrete
route instead: a random walk on the flip graph of matrix multiplication
schemes (search.c; Kauers and Moosbauer, ISSAC 2023) from the classical
scheme down to rank R.

* over Z (the default): the walk itself keeps every coefficient in
  {-1, 0, 1}; each of its moves is an identity over the integers, so every
  scheme it reaches is an exact algorithm;
* over GF(2) (--over gf2): the walk runs modulo 2 and each scheme is then
  lifted to coefficients in {-1, 0, 1}: every non-zero GF(2) coefficient x
  becomes 1 + 2 d with d in {0, 1}; modulo 4 the Brent equations
  (Equation (2)) are linear in the d's over GF(2): for each (i, j, k) the
  terms r with u_ir v_jr w_kr != 0 must satisfy
  sum_r (d(u_ir) + d(v_jr) + d(w_kr)) = (T_ijk - #terms) / 2 (mod 2);
  solutions of that system (a particular one plus seeded random combinations
  of the null space) are tried until one satisfies the equations over the
  integers.  Many GF(2) schemes have no such lift.

The exact Brent check is the only acceptance gate.  Among the accepted
schemes of all seeds the one with the fewest non-zero coefficients is kept
(fewer non-zeros: fewer operand and product reads in the addition passes and
less rounding-error growth, Section 6).  The walk is deterministic for a
given seed, so the command line recorded in a table's header regenerates it.

    python paper_1409_2908_amd/algorithms/search.py M K N R --seeds 1-8 \\
        [--count 4] [--flips N] [--plateau N] [--over z|gf2] [--out FILE]

prints the table (the text format gen_tables.py reads) or writes it to FILE
with the command line that regenerates it.
"""
import argparse
import os
import random
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(os.path.dirname(HERE), "_build")


def build_walker():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "flip_search")
    src = os.path.join(HERE, "search.c")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-o", exe, src])
    return exe


def tensor_entry(M, K, N, i, j, k):
    ia, ib = divmod(i, K)
    jb, jc = divmod(j, N)
    ka, kc = divmod(k, N)
    return 1 if (ib == jb and jc == kc and ia == ka) else 0


def brent_exact(M, K, N, U, V, W):
    """Sum_r U[i][r] V[j][r] W[k][r] == T_ijk for every (i, j, k), in integers."""
    R = len(U[0])
    for i in range(M * K):
        for j in range(K * N):
            uv = [U[i][r] * V[j][r] for r in range(R)]
            if not any(uv):
                if any(tensor_entry(M, K, N, i, j, k) for k in range(M * N)):
                    return False
                continue
            for k in range(M * N):
                if sum(uv[r] * W[k][r] for r in range(R)) != tensor_entry(M, K, N, i, j, k):
                    return False
    return True


def run_walk(exe, M, K, N, R, seed, flips, plateau, count, over="gf2"):
    """Schemes from the walker.  GF(2): lists of (u, v, w) bit masks.  Z:
    (U, V, W) coefficient matrices (MK x R, KN x R, MN x R)."""
    args = [exe, str(M), str(K), str(N), str(R), str(seed), str(flips), str(plateau), str(count)]
    if over == "z":
        args.append("z")
    p = subprocess.run(args, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    out = []
    val = {"n": -1, "0": 0, "1": 1}
    for line in p.stdout.splitlines():
        t = line.split()
        r = int(t[0])
        if over == "z":
            U = [[0] * r for _ in range(M * K)]
            V = [[0] * r for _ in range(K * N)]
            W = [[0] * r for _ in range(M * N)]
            for q in range(r):
                for X, txt in ((U, t[1 + 3 * q]), (V, t[2 + 3 * q]), (W, t[3 + 3 * q])):
                    assert len(txt) == len(X)
                    for i, ch in enumerate(txt):
                        X[i][q] = val[ch]
            out.append((U, V, W))
        else:
            masks = [int(x, 16) for x in t[1:]]
            out.append([(masks[3 * q], masks[3 * q + 1], masks[3 * q + 2]) for q in range(r)])
    return out


def _solve_gf2(rows, nvars):
    """rows: (bitmask over variables, rhs bit).  Returns (particular solution
    as a bitmask, null space basis as bitmasks) or None if inconsistent."""
    pivots = {}  # pivot column -> (mask, rhs)
    for mask, rhs in rows:
        for col, (pm, pr) in pivots.items():
            if (mask >> col) & 1:
                mask ^= pm
                rhs ^= pr
        if mask == 0:
            if rhs:
                return None
            continue
        col = mask.bit_length() - 1
        for c2 in list(pivots):
            pm, pr = pivots[c2]
            if (pm >> col) & 1:
                pivots[c2] = (pm ^ mask, pr ^ rhs)
        pivots[col] = (mask, rhs)
    sol = 0
    for col, (pm, pr) in pivots.items():
        if pr:
            sol |= 1 << col
    free = [c for c in range(nvars) if c not in pivots]
    basis = []
    for f in free:
        vec = 1 << f
        for col, (pm, pr) in pivots.items():
            if (pm >> f) & 1:
                vec |= 1 << col
        basis.append(vec)
    return sol, basis


def lift(M, K, N, scheme, rng, tries=400):
    """Integer coefficients in {-1, 0, 1} on the scheme's support satisfying
    the Brent equations exactly, or None."""
    R = len(scheme)
    MK, KN, MN = M * K, K * N, M * N
    var = {}  # (side, row, r) -> variable index
    for r, (u, v, w) in enumerate(scheme):
        for side, mask, n in ((0, u, MK), (1, v, KN), (2, w, MN)):
            for x in range(n):
                if (mask >> x) & 1:
                    var[(side, x, r)] = len(var)
    rows = []
    for i in range(MK):
        for j in range(KN):
            for k in range(MN):
                terms = [r for r, (u, v, w) in enumerate(scheme) if (u >> i) & (v >> j) & (w >> k) & 1]
                if not terms:
                    continue
                t = tensor_entry(M, K, N, i, j, k)
                mask = 0
                for r in terms:
                    mask ^= (1 << var[(0, i, r)]) ^ (1 << var[(1, j, r)]) ^ (1 << var[(2, k, r)])
                rows.append((mask, ((t - len(terms)) // 2) & 1))
    solved = _solve_gf2(rows, len(var))
    if solved is None:
        return None
    sol, basis = solved
    for attempt in range(tries):
        d = sol
        if attempt:
            for b in basis:
                if rng.random() < 0.5:
                    d ^= b
        U = [[0] * R for _ in range(MK)]
        V = [[0] * R for _ in range(KN)]
        W = [[0] * R for _ in range(MN)]
        for (side, x, r), idx in var.items():
            val = -1 if (d >> idx) & 1 else 1
            (U, V, W)[side][x][r] = val
        if brent_exact(M, K, N, U, V, W):
            return U, V, W
    return None


def lift_2adic(M, K, N, scheme, bits=24, bound=4):
    """Integer coefficients for a GF(2) scheme by Hensel lifting, every entry
    free (not only the signs on the GF(2) support), or None.

    A solution x modulo 2^e of the Brent equations F(x) = 0 (Equation (2))
    extends to x + 2^e y modulo 2^(e+1) exactly when J y = -F(x) / 2^e
    (mod 2), where J is the Jacobian of F at the GF(2) scheme (the same
    matrix at every step).  Each step takes the solution with the free
    variables zero, entries outside the GF(2) support chosen free first, so
    the lift stays as close to the support as the equations allow.  After
    `bits` steps the balanced residues are taken as integers; they are
    returned when every one is at most `bound` in magnitude and the exact
    Brent check passes."""
    R = len(scheme)
    sizes = (M * K, K * N, M * N)
    keys = [(s, x, r) for s in range(3) for x in range(sizes[s]) for r in range(R)]
    bit = {key: (scheme[key[2]][key[0]] >> key[1]) & 1 for key in keys}
    order = sorted(keys, key=lambda key: bit[key])  # off-support first: low columns, free if possible
    col = {key: c for c, key in enumerate(order)}
    eqs = [(i, j, k) for i in range(sizes[0]) for j in range(sizes[1]) for k in range(sizes[2])]
    rows = []
    for (i, j, k) in eqs:
        mask = 0
        for r in range(R):
            u, v, w = bit[(0, i, r)], bit[(1, j, r)], bit[(2, k, r)]
            if v & w:
                mask ^= 1 << col[(0, i, r)]
            if u & w:
                mask ^= 1 << col[(1, j, r)]
            if u & v:
                mask ^= 1 << col[(2, k, r)]
        rows.append(mask)
    # Gauss-Jordan once, recording which equations each pivot row sums, so
    # that every step only needs parities of the new right-hand side
    piv = {}
    zero_rows = []
    for e, mask in enumerate(rows):
        comb = 1 << e
        for c, (pm, pc) in piv.items():
            if (mask >> c) & 1:
                mask ^= pm
                comb ^= pc
        if mask == 0:
            zero_rows.append(comb)
            continue
        top = mask.bit_length() - 1
        for c in list(piv):
            pm, pc = piv[c]
            if (pm >> top) & 1:
                piv[c] = (pm ^ mask, pc ^ comb)
        piv[top] = (mask, comb)
    X = [[[bit[(s, x, r)] for r in range(R)] for x in range(sizes[s])] for s in range(3)]
    T = [tensor_entry(M, K, N, i, j, k) for (i, j, k) in eqs]
    mod = 2
    for _ in range(1, bits):
        rhs = 0
        for e, ((i, j, k), t) in enumerate(zip(eqs, T)):
            a, b, c = X[0][i], X[1][j], X[2][k]
            f = sum(a[r] * b[r] * c[r] for r in range(R)) - t
            if (f // mod) & 1:
                rhs |= 1 << e
        if any(bin(z & rhs).count("1") & 1 for z in zero_rows):
            return None
        for c, (pm, pc) in piv.items():
            if bin(pc & rhs).count("1") & 1:
                s, x, r = order[c]
                X[s][x][r] += mod
        mod *= 2
        for Xs in X:
            for row in Xs:
                for r in range(R):
                    v = row[r] % mod
                    row[r] = v - mod if v >= mod // 2 else v
    if max(abs(v) for Xs in X for row in Xs for v in row) > bound:
        return None
    U, V, W = X
    return (U, V, W) if brent_exact(M, K, N, U, V, W) else None


def nnz(U, V, W):
    return sum(1 for X in (U, V, W) for row in X for x in row if x)


def canonical(U, V, W):
    """Terms sorted, so equal schemes print equally (the order of the products
    does not change the algorithm)."""
    R = len(U[0])
    cols = sorted(range(R), key=lambda r: ([U[i][r] for i in range(len(U))], [V[j][r] for j in range(len(V))],
                                            [W[k][r] for k in range(len(W))]), reverse=True)
    return ([[row[r] for r in cols] for row in U], [[row[r] for r in cols] for row in V],
            [[row[r] for r in cols] for row in W])


def search(M, K, N, R, seeds, count=4, flips=10 ** 10, plateau=50000, over="z", log=sys.stderr,
           lift_mode="sign"):
    exe = build_walker()
    best = None
    for seed in seeds:
        rng = random.Random(seed)
        for scheme in run_walk(exe, M, K, N, R, seed, flips, plateau, count, over):
            if over == "z":
                U, V, W = scheme
            else:
                lifted = lift(M, K, N, scheme, rng)
                if lifted is None and lift_mode == "2adic":
                    lifted = lift_2adic(M, K, N, scheme)
                if lifted is None:
                    print(f"seed {seed}: a rank-{len(scheme)} scheme did not lift", file=log)
                    continue
                U, V, W = lifted
            rank = len(U[0])
            if not brent_exact(M, K, N, U, V, W):
                raise RuntimeError(f"seed {seed}: the walker returned a scheme that fails the Brent equations")
            z = nnz(U, V, W)
            print(f"seed {seed}: rank {rank}, {z} non-zeros", file=log)
            if rank == R and (best is None or z < best[0]):
                best = (z, seed, canonical(U, V, W))
    return best


def format_table(M, K, N, R, U, V, W, header):
    lines = [f"# {h}" for h in header]
    lines.append(f"{M} {K} {N} {R}")
    for X in (U, V, W):
        for row in X:
            lines.append(" ".join(str(x) for x in row))
    return "\n".join(lines) + "\n"


def _seeds(text):
    out = []
    for part in text.split(","):
        if "-" in part:
            a, b = part.split("-")
            out += list(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("M", type=int)
    ap.add_argument("K", type=int)
    ap.add_argument("N", type=int)
    ap.add_argument("R", type=int)
    ap.add_argument("--seeds", default="1-4")
    ap.add_argument("--count", type=int, default=4, help="schemes per seed")
    ap.add_argument("--flips", type=int, default=10 ** 10, help="flip budget per seed")
    ap.add_argument("--plateau", type=int, default=50000, help="flips without a reduction before a plus step")
    ap.add_argument("--over", choices=("z", "gf2"), default="z", help="walk over the integers or GF(2)")
    ap.add_argument("--lift", choices=("sign", "2adic"), default="sign",
                    help="GF(2) schemes: signs on the support only, or also the 2-adic lift of every entry")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    best = search(args.M, args.K, args.N, args.R, _seeds(args.seeds), args.count, args.flips, args.plateau,
                  args.over, lift_mode=args.lift)
    if best is None:
        print("no scheme of that rank was found and lifted", file=sys.stderr)
        return 1
    z, seed, (U, V, W) = best
    name = f"fmm_{args.M}{args.K}{args.N}_{args.R}"
    cmd = (f"python paper_1409_2908_amd/algorithms/search.py {args.M} {args.K} {args.N} {args.R} "
           f"--seeds {args.seeds} --count {args.count} --flips {args.flips} --plateau {args.plateau} "
           f"--over {args.over}" + (" --lift 2adic" if args.lift == "2adic" else ""))
    how = ("over the integers with coefficients in {-1,0,1}" if args.over == "z" else
           "over GF(2), lifted to coefficients in {-1,0,1} (Brent equations mod 4 as a GF(2) linear system)"
           if args.lift == "sign" else
           "over GF(2), lifted to integers (signs on the support first, else a 2-adic lift of every entry)")
    header = [f"<{args.M},{args.K},{args.N};{args.R}> {name}",
              "Found by a random walk on the flip graph (Kauers and Moosbauer, ISSAC 2023) from the classical",
              f"scheme, {how},",
              f"accepted by the exact Brent check; {z} non-zeros (the sparsest of the seeds', from seed {seed}).",
              f"Regenerate: {cmd}",
              "Format: 'M K N R', then MK rows of U, KN rows of V, MN rows of W (R entries each)."]
    text = format_table(args.M, args.K, args.N, args.R, U, V, W, header)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    else:
        sys.stdout.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
