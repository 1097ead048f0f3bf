"""Writes tests/golden/permutation_vectors.txt from the CPU oracle only.

Each line: n seed t followed by sigma_t(p) for p = 0 .. min(n, 64) - 1 and,
for n > 64, the positions n-8 .. n-1 after a '|' separator.
Run: python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.permutation import sweep_permutation  # noqa: E402

CASES = [
    (1, 0, 0), (2, 0, 0), (3, 7, 1), (4, 1, 2), (5, 123, 0), (16, 101, 0),
    (16, 101, 1), (17, 5, 9), (64, 101, 0), (64, 101, 1), (64, 102, 0),
    (100, 2**63 + 11, 2**40 + 3), (1000, 42, 7), (8192, 102, 0),
    (8192, 102, 1234), (65537, 9, 5), (1_000_000, 103, 0),
]


def main():
    lines = ["# sigma_t(p) of the sweep order (oracle/permutation.py); written by make_golden.py"]
    for n, seed, t in CASES:
        s = sweep_permutation(n, seed, t)
        head = " ".join(str(int(v)) for v in s[:64])
        line = "%d %d %d  %s" % (n, seed, t, head)
        if n > 64:
            line += " | " + " ".join(str(int(v)) for v in s[n - 8:])
        lines.append(line)
    with open(os.path.join(HERE, "permutation_vectors.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
