"""The two constant tables of the path generator's binary64 math, from their
definitions at 60 significant digits (Python's decimal module), each entry
rounded once to binary64:

  kLogTab[j] = log(1/2 + j/128 + 1/256),  j = 0..63   (Tang's logarithm)
  kExpTab[j] = 2^(j/64),                   j = 0..63   (Tang's exponential)

    python gen_math_tables.py           print both tables as C initialisers
    python gen_math_tables.py --check   compare them with amq_kernels.hip
                                        (exit status 1 on any difference)
"""
import os
import re
import sys
from decimal import Decimal, getcontext

getcontext().prec = 60
HERE = os.path.dirname(os.path.abspath(__file__))


def log_table():
    return [float((Decimal(1) / 2 + Decimal(j) / 128 + Decimal(1) / 256).ln()) for j in range(64)]


def exp_table():
    ln2 = Decimal(2).ln()
    return [float((ln2 * j / 64).exp()) for j in range(64)]


def c_rows(vals):
    hx = [v.hex() for v in vals]
    return "\n".join("    " + ", ".join(hx[i:i + 4]) + "," for i in range(0, len(hx), 4))


def source_table(name):
    text = open(os.path.join(HERE, "amq_kernels.hip")).read()
    m = re.search(r"__constant__ double " + name + r"\[64\] = \{(.*?)\};", text, re.S)
    if not m:
        raise SystemExit(f"{name} not found in amq_kernels.hip")
    return [float.fromhex(t) for t in re.findall(r"-?0x[0-9a-fA-Fp.+-]+", m.group(1))]


def main(argv):
    tables = {"kLogTab": log_table(), "kExpTab": exp_table()}
    if "--check" in argv:
        bad = [n for n, v in tables.items() if source_table(n) != v]
        for n in bad:
            print(f"{n} differs from its definition")
        return 1 if bad else 0
    for n, v in tables.items():
        print(f"__constant__ double {n}[64] = {{\n{c_rows(v)}\n}};")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
