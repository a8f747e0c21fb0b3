"""Hand-worked rule scenarios: parsing of the fixtures in tests/golden/.

A grid is a list of row strings of space-separated cell tokens:

    P-:0   plain, neutral, army 0        P0:5   plain owned by player 0, army 5
    M      mountain (neutral, army 0)    C-:45  neutral castle (city) with 45
    G1:3   general of player 1, army 3   C0:7   castle owned by player 0

The general positions (gpos) come from the G tokens of a scenario's initial
grid (token owner = player) unless the scenario lists "gpos" itself.  This
module only converts text to the public host-state arrays and back; it holds
none of the game's rules.
"""
from __future__ import annotations

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_TYPES = {"P": 0, "M": 1, "C": 2, "G": 3}
_NAMES = {v: k for k, v in _TYPES.items()}


def parse_cell(tok: str):
    if tok == "M":
        return 1, -1, 0
    t = _TYPES[tok[0]]
    o, a = tok[1:].split(":")
    return t, (-1 if o == "-" else int(o)), int(a)


def parse_grid(rows):
    cells = [parse_cell(t) for r in rows for t in r.split()]
    H, W = len(rows), len(rows[0].split())
    typ = np.array([c[0] for c in cells], np.uint8)
    own = np.array([c[1] for c in cells], np.int8)
    army = np.array([c[2] for c in cells], np.int32)
    return H, W, typ, own, army


def format_grid(H, W, typ, own, army):
    rows = []
    for r in range(H):
        toks = []
        for c in range(W):
            i = r * W + c
            if typ[i] == 1 and own[i] == -1 and army[i] == 0:
                toks.append("M")
            else:
                o = "-" if own[i] < 0 else str(int(own[i]))
                toks.append(f"{_NAMES[int(typ[i])]}{o}:{int(army[i])}")
        rows.append(" ".join(toks))
    return rows


def load(name: str = "scenarios.json"):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)["scenarios"]


def initial_state(sc: dict) -> dict:
    """Host state (E=1) of a scenario's initial grid."""
    H, W, typ, own, army = parse_grid(sc["grid"])
    P = sc["P"]
    if "gpos" in sc:
        gpos = np.array(sc["gpos"], np.int16)
    else:
        gpos = np.full(P, -1, np.int16)
        for i in range(H * W):
            if typ[i] == 3:
                gpos[own[i]] = i
    assert (gpos >= 0).all(), "every player needs a general"
    alive = sc.get("alive", (1 << P) - 1)
    return {
        "owner": own.reshape(1, -1).copy(), "army": army.reshape(1, -1).copy(),
        "type": typ.reshape(1, -1).copy(), "turn": np.array([sc["turn"]], np.int32),
        "episode": np.array([sc.get("episode", 0)], np.uint32),
        "alive": np.array([alive], np.uint8), "finished": np.array([0], np.uint8),
        "gpos": gpos.reshape(1, -1).copy(),
    }


def encode_actions(sc_step: dict, P: int) -> np.ndarray:
    """Actions of one scenario step: "pass", an integer, or [cell, k]."""
    out = np.zeros((1, P), np.int32)
    for p, a in enumerate(sc_step["actions"]):
        if a == "pass":
            out[0, p] = 0
        elif isinstance(a, list):
            out[0, p] = a[0] * 9 + a[1]
        else:
            out[0, p] = int(a)
    return out


def grid_of(st: dict, H: int, W: int):
    return format_grid(H, W, st["type"][0], st["owner"][0], st["army"][0])
