"""Parser for tests/golden/hand_examples.txt (hand-worked cases)."""
import ipaddress
import os
from collections import defaultdict

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_examples.txt")


def ip(s: str) -> int:
    return int(ipaddress.IPv4Address(s))


def cidr(s: str):
    a, z = s.split("/")
    return ip(a), int(z)


def load():
    g = defaultdict(list)
    tables = defaultdict(lambda: ([], [], []))
    with open(PATH) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            t = line.split()
            k = t[0]
            if k == "mask":
                g["mask"].append((int(t[1]), int(t[2], 16)))
            elif k == "match":
                b, z = cidr(t[2])
                g["match"].append((ip(t[1]), b, z, int(t[3], 16), int(t[4])))
            elif k == "table":
                b, z = cidr(t[2])
                tb = tables[t[1]]
                tb[0].append(b)
                tb[1].append(z)
                tb[2].append(int(t[3]))
            elif k == "lpm":
                g["lpm"].append((t[1], ip(t[2]), None if t[3] == "NONE" else int(t[3])))
            elif k == "ends":
                g["ends"].append((t[1], [int(x, 16) for x in t[2].split(",")],
                                  [int(x) for x in t[3].split(",")]))
            elif k == "pos":
                g["pos"].append((t[1], ip(t[2]), int(t[3])))
            elif k == "label":
                g["label"].append((t[1], ip(t[2]), ip(t[3]), int(t[4])))
            elif k == "bin":
                g["bin"].append((int(t[1]), int(t[2]), int(t[3]), int(t[4]),
                                 None if t[5] == "DROP" else int(t[5])))
            elif k == "sess":
                g["sess"].append((int(t[1]), int(t[2]), int(t[3])))
            elif k == "hist":
                i = t.index(":")
                g["hist"].append((int(t[1]), int(t[2]), int(t[3]),
                                  int(t[i + 1]), int(t[i + 2]), int(t[i + 3]), int(t[i + 4])))
            elif k == "drop":
                g["drop"].append((int(t[1]), int(t[2]), int(t[3])))
            else:
                raise ValueError(line)
    return g, dict(tables)
