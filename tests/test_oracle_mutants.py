"""Planted mistakes in copies of the oracle must each fail at least one pin.

Every mutant is a one-token change of the kind a careless edit makes: a
flipped comparison, a swapped operand, a dropped term, an off-by-one.  The
real ``oracle.c`` is never modified; each mutant is compiled from a patched
copy into a temporary directory, on the CPU.
"""
import multiprocessing
import os
import shutil
import subprocess

import pytest

from tests import oracle_pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "collinear-kept": ("<= 0) --t;", "< 0) --t;"),
    "min-as-max": ("if (y < lo[c]) lo[c] = y;", "if (y > lo[c]) lo[c] = y;"),
    "max-as-min": ("if (y > hi[c]) hi[c] = y;", "if (y < hi[c]) hi[c] = y;"),
    "sentinel-lo": ("lo[c] = q + 1;", "lo[c] = q;"),
    "sentinel-from-p": ("lo[c] = q + 1;", "lo[c] = p + 1;"),
    "sentinel-hi": ("hi[c] = -1;", "hi[c] = 0;"),
    "x-y-swapped": ("const int32_t c = pts[2 * j] - 1, y = pts[2 * j + 1];",
                    "const int32_t c = pts[2 * j + 1] - 1, y = pts[2 * j];"),
    "store-lo-into-hi": ("if (y > hi[c]) hi[c] = y;", "if (y > hi[c]) hi[c] = lo[c];"),
    "cross-sign": ("return (ax - ox) * (by - oy) - (ay - oy) * (bx - ox);",
                   "return (ay - oy) * (bx - ox) - (ax - ox) * (by - oy);"),
    "cross-dropped-term": ("return (ax - ox) * (by - oy) - (ay - oy) * (bx - ox);",
                           "return (ax - ox) * (by - oy);"),
    "cross-transposed": ("return (ax - ox) * (by - oy) - (ay - oy) * (bx - ox);",
                         "return (ax - ox) * (by - oy) - (ay - oy) * (bx - oy);"),
    "keep-last-of-lower": ("    for (int64_t i = 0; i + 1 < t; ++i) {\n        vx[h] = sx[i];",
                           "    for (int64_t i = 0; i < t; ++i) {\n        vx[h] = sx[i];"),
    "mask-bit-off-by-one": ("M[c / 64] |= (uint64_t)1 << (c % 64);", "M[c / 64] |= (uint64_t)1 << ((c + 1) % 64);"),
    "ctz-pos-off-by-one": ("pos[c++] = or_ctz64(w);", "pos[c++] = or_ctz64(w) + 1;"),
    "ctz-clears-two-bits": ("w &= w - 1) pos", "w &= w - 2) pos"),
    "valid-inverted": ("return !(lo == q + 1 && hi == -1);", "return (lo == q + 1 && hi == -1);"),
    "reduced-repeats-single": ("if (chi[t] > clo[t]) {", "if (chi[t] >= clo[t]) {"),
    "range-check-off": ("if (x < 1 || x > p || y < 1 || y > q) return OR_ERANGE;",
                        "if (x < 1 || x > p || y < 1) return OR_ERANGE;"),
    "range-check-y-against-p": ("if (x < 1 || x > p || y < 1 || y > q) return OR_ERANGE;",
                                "if (x < 1 || x > p || y < 1 || y > p) return OR_ERANGE;"),
    "bbox-ymin-from-x": ("if (y < ymin) ymin = y;", "if (x < ymin) ymin = x;"),
    "translate-off-by-one": ("out[2 * j] = (int32_t)((int64_t)pts[2 * j] - box[0] + 1);",
                             "out[2 * j] = (int32_t)((int64_t)pts[2 * j] - box[0]);"),
    "side-from-x-only": ("int64_t side = ex > ey ? ex : ey;", "int64_t side = ex;"),
    "tree-bit-not-shifted": ("            bit >>= 6;                          /* the word index becomes the bit index above */",
                             "            bit >>= 5;                          /* the word index becomes the bit index above */"),
    "tree-child-index": ("int64_t child = word * 64 + pos[t];", "int64_t child = word * 63 + pos[t];"),
    "tree-one-level-short": ("        if (words == 1) break;\n        words = (words + 63) / 64;",
                             "        words = (words + 63) / 64;\n        if (words == 1) break;"),
    "melkman-skip-either-side": ("if (or_orient(DQ(top - 1), DQ(top), v) > 0 && or_orient(DQ(bot), DQ(bot + 1), v) > 0) continue;",
                                 "if (or_orient(DQ(top - 1), DQ(top), v) > 0 || or_orient(DQ(bot), DQ(bot + 1), v) > 0) continue;"),
    "melkman-clockwise-start": ("or_orient(a, b, c) > 0 ? a : b;", "or_orient(a, b, c) < 0 ? a : b;"),
    "melkman-orient-term": ("return abx * acy - aby * acx;", "return abx * acy - aby * acy;"),
    "scale-rounds-up": ("double t = floor(((double)v - o) * s);", "double t = ceil(((double)v - o) * s);"),
    "scale-origin-added": ("double t = floor(((double)v - o) * s);", "double t = floor(((double)v + o) * s);"),
    "float-box-keeps-nan": ("if (x != x || y != y) continue;", "if (x != x) continue;"),
    "chain-skips-last": ("for (int32_t c = 0; c < p; ++c) {\n        if (!or_valid(lo[c], hi[c], q)) continue;\n        x[k] = c + 1;",
                         "for (int32_t c = 0; c + 1 < p; ++c) {\n        if (!or_valid(lo[c], hi[c], q)) continue;\n        x[k] = c + 1;"),
    "rect-rows-from-columns": ("*q = (int32_t)ey;", "*q = (int32_t)ex;"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(old) >= 1, f"mutant {name}: pattern not found"
    src = src.replace(old, new)
    d = tmp_path / name
    d.mkdir()
    shutil.copy(os.path.join(ROOT, "oracle", "oracle.h"), d / "oracle.h")
    (d / "oracle.c").write_text(src)
    out = d / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(out),
                    str(d / "oracle.c"), "-lm"],
                   check=True)
    return str(out)


def _pins_catch(lib: str) -> None:
    """Child process: exit 0 as soon as a pin fails on ``lib``, 1 if none does."""
    for pin in oracle_pins.FAST_PINS + [p for p in oracle_pins.ALL_PINS if p not in oracle_pins.FAST_PINS]:
        if pin(lib):
            os._exit(0)
    os._exit(1)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)
    # a mutant that writes out of bounds may crash the process that runs it:
    # the pins run in a child process (forked from a clean single-threaded
    # server, never from this possibly multi-threaded one), and a crash
    # counts as a catch
    proc = multiprocessing.get_context("forkserver").Process(target=_pins_catch, args=(lib,))
    proc.start()
    proc.join(300)
    if proc.is_alive():
        proc.kill()
        proc.join()
        pytest.fail(f"pins on mutant {name} did not finish")
    assert proc.exitcode != 1, f"no pin catches mutant {name}"
