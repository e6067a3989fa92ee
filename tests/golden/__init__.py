"""Loader for the small text fixtures in this folder.

Each fixture line is `key=value` pairs separated by `;`.  Values are numbers,
vectors `[a,b,c]`, or arithmetic with sqrt/inf written out by hand from the
closed form that the line's comment derives.
"""
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_NS = {"sqrt": math.sqrt, "inf": math.inf, "__builtins__": {}}


def load_golden(name):
    out = []
    with open(os.path.join(_HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            rec = {}
            for item in line.split(";"):
                k, v = item.split("=", 1)
                rec[k.strip()] = eval(v.strip(), _NS)  # fixture values written in this repo
            out.append(rec)
    return out
