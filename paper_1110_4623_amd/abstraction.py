"""Machine abstraction of Section 4, computed from the memory-system tests of Section 3.

The twelve tests (Table 1) time one thousand accesses by each workgroup's master thread:
contentious (every workgroup on one word) or noncontentious (own word, own line), volatile
or atomic, read or write, and the volatile tests again after one initial atomic.  From the
times the paper derives the ratios of Table 2 (contentious : noncontentious) and Table 3
(each access kind : the volatile access of the same contention), and classifies a GPU by
three parameters:

* Atomic:Volatile ratio -- whether designs that spin with atomics are viable;
* Contentious:Noncontentious volatile ratio -- how well polling ("sleeping") performs;
* whether an atomic unit with a non-empty queue holds a line hostage -- whether volatile
  polling of a word that receives atomics is slowed down (volatile-after-atomic : volatile).

`tables` and `card` work on any times (the paper's own Table 1 included); `measure` runs
the twelve tests on this GPU through libsp.
"""

from __future__ import annotations

KINDS = ["vol", "atom", "vol_after_atom"]
COLUMNS = ["read", "write"]


def _key(contentious: bool, kind: str, col: str) -> str:
    return f"{'cont' if contentious else 'noncont'}_{kind}_{col}"


def tables(times: dict) -> tuple[dict, dict]:
    """times[key] for key in {cont,noncont}_{vol,atom,vol_after_atom}_{read,write}.

    Returns (table2, table3):
      table2[kind][col] = contentious time / noncontentious time (Table 2);
      table3[(contention, kind)][col] = time / volatile time of the same contention, for
      kind in atom and vol_after_atom (Table 3)."""
    t2 = {k: {c: times[_key(True, k, c)] / times[_key(False, k, c)] for c in COLUMNS}
          for k in KINDS}
    t3 = {}
    for cont in (True, False):
        for k in ("atom", "vol_after_atom"):
            t3[("cont" if cont else "noncont", k)] = {
                c: times[_key(cont, k, c)] / times[_key(cont, "vol", c)] for c in COLUMNS}
    return t2, t3


def card(times: dict, hostage_threshold: float = 1.5) -> dict:
    """The three parameters of Section 4 plus the derived per-access rates."""
    t2, t3 = tables(times)
    hostage = {c: t3[("cont", "vol_after_atom")][c] for c in COLUMNS}
    return {
        "atomic_to_volatile": {c: t3[("cont", "atom")][c] for c in COLUMNS},
        "atomic_to_volatile_noncontentious": {c: t3[("noncont", "atom")][c] for c in COLUMNS},
        "contentious_to_noncontentious_volatile": dict(t2["vol"]),
        "contentious_to_noncontentious_atomic": dict(t2["atom"]),
        "volatile_after_atomic_to_volatile": hostage,
        "atomic_unit_holds_line_hostage": {c: hostage[c] > hostage_threshold for c in COLUMNS},
        "table2": {k: dict(v) for k, v in t2.items()},
        "table3": {f"{a}_{b}": dict(v) for (a, b), v in t3.items()},
    }


_TEST_OF_KEY = {
    "cont_vol_read": "cont_vol_read", "cont_vol_write": "cont_vol_write",
    "noncont_vol_read": "noncont_vol_read", "noncont_vol_write": "noncont_vol_write",
    "cont_atom_read": "cont_atom_read", "cont_atom_write": "cont_atom_write",
    "noncont_atom_read": "noncont_atom_read", "noncont_atom_write": "noncont_atom_write",
    "cont_vol_after_atom_read": "cont_vol_read_after_atom",
    "cont_vol_after_atom_write": "cont_vol_write_after_atom",
    "noncont_vol_after_atom_read": "noncont_vol_read_after_atom",
    "noncont_vol_after_atom_write": "noncont_vol_write_after_atom",
}


def measure(ctx, nwg: int, n_ops: int = 1000, stride: int = 256, reps: int = 3) -> dict:
    """Kernel times (ms, best of `reps`) of the twelve tests with `nwg` workgroups."""
    from . import api
    times = {}
    for key, test in _TEST_OF_KEY.items():
        best = None
        for _ in range(reps):
            _, _, st = api.paper12(ctx, test, nwg=nwg, lanes=64, n_ops=n_ops, stride=stride)
            best = st["kernel_ms"] if best is None else min(best, st["kernel_ms"])
        times[key] = best
    return times


def paper_table1_times(column_index: int, table1: dict) -> dict:
    """Map one column of the paper's Table 1 (as stored in tests/golden) to `times` keys
    with both read and write entries taken from the matching read/write columns."""
    rows = {"contentious_volatile": ("cont", "vol"),
            "noncontentious_volatile": ("noncont", "vol"),
            "contentious_atomic": ("cont", "atom"),
            "noncontentious_atomic": ("noncont", "atom"),
            "contentious_volatile_after_atomic": ("cont", "vol_after_atom"),
            "noncontentious_volatile_after_atomic": ("noncont", "vol_after_atom")}
    times = {}
    for row, (cont, kind) in rows.items():
        times[f"{cont}_{kind}_read"] = table1[row][column_index]
        times[f"{cont}_{kind}_write"] = table1[row][column_index + 1]
    return times
