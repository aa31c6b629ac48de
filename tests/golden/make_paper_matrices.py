"""Writes paper_matrices.txt: the fixed test matrices of the paper's
benchmark section (Sec. 3), A = [sqrt5 (i + j - 1)] and B = [sqrt3 (n - i)]
for i, j = 1..n, and their product C = A B, whose entries are
C_ij = sqrt15 * N_i with the integer N_i = sum_l (i + l - 1)(n - l).

Only exact integer arithmetic: every entry is stored as an integer
coefficient of sqrt5, sqrt3 or sqrt15.  Run from the repository root:
    python tests/golden/make_paper_matrices.py
"""
import os

SIZES = (1, 2, 4, 7, 32)


def lines():
    out = ["# Sec. 3 fixed matrices: A_ij = sqrt(5) * a_ij, B_ij = sqrt(3) * b_ij, (A B)_ij = sqrt(15) * c_ij",
           "# one line per n: 'n <n>', then 'A', 'B', 'C' rows of integer coefficients (i = 1..n, j = 1..n)"]
    for n in SIZES:
        a = [[i + j - 1 for j in range(1, n + 1)] for i in range(1, n + 1)]
        b = [[n - i for j in range(1, n + 1)] for i in range(1, n + 1)]
        c = [[sum(a[i][l] * b[l][j] for l in range(n)) for j in range(n)] for i in range(n)]
        out.append(f"n {n}")
        for name, M in (("A", a), ("B", b), ("C", c)):
            for row in M:
                out.append(name + " " + " ".join(str(v) for v in row))
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_matrices.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines()) + "\n")
    print("wrote", path)
