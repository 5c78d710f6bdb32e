"""Write op_counts.txt from the closed forms of Sections 2.2 and 2.3.

For order n = 2^k and recursion down to 1x1 blocks:
  Strassen  7 n^{log2 7} - 6 n^2 = 7 * 7^k - 6 * 4^k     (Section 2.2)
  Winograd  6 n^{log2 7} - 5 n^2 = 6 * 7^k - 5 * 4^k     (same recurrence,
                                                          15 additions/level)
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    lines = ["# k  n=2^k  strassen_ops  winograd_ops  (multiplications + additions)"]
    for k in range(1, 8):
        lines.append(f"{k} {2**k} {7 * 7**k - 6 * 4**k} {6 * 7**k - 5 * 4**k}")
    with open(os.path.join(HERE, "op_counts.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
