"""Writes laplace_sigma0.txt from the sine-series closed form (no solver)."""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def closed_form(n):
    h = 1.0 / n
    s = math.fsum(
        (1.0 / math.tan(p * math.pi * h / 2)) ** 2 * (1.0 / math.tan(q * math.pi * h / 2)) ** 2
        / (math.sin(p * math.pi * h / 2) ** 2 + math.sin(q * math.pi * h / 2) ** 2)
        for p in range(1, n, 2) for q in range(1, n, 2))
    return h ** 6 * s


if __name__ == "__main__":
    path = os.path.join(HERE, "laplace_sigma0.txt")
    head = [l for l in open(path) if l.startswith("#")]
    with open(path, "w") as f:
        f.writelines(head)
        for n in (4, 8, 16, 32, 64, 128, 256):
            f.write("%d %.17g\n" % (n, closed_form(n)))
