"""Instantiation table of the solve kernel: for every lanes-per-column L, the
entries-per-lane E that are compiled (a rank r runs on the smallest listed E
with E * L >= r).  ``generate()`` writes the per-L instantiation sources and
the table header under ``csrc/``; build.py calls it before compiling, and it
rewrites a file only when its text changes.
"""
from __future__ import annotations

import os

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# L: E values.  Small E for wide groups (few columns, latency-bound launches),
# a fine grid around the common ranks for the throughput layouts.
VARIANTS = {
    1: [1, 2, 4, 6, 8, 12, 16, 20, 24, 28, 32],
    2: [2, 4, 6, 8, 12, 16, 20, 24, 28, 32],
    4: [1, 2, 4, 6, 8, 12, 16, 18, 20, 22, 24, 25, 26, 28, 30, 32],
    8: [1, 2, 3, 4, 6, 8, 10, 12, 13, 16],
    16: [1, 2, 3, 4, 5, 6, 7, 8],
}

_SOLO = """// Solve-kernel instantiations with {L} lane(s) per column (nqp_kernel.h).
// Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {{

hipError_t launch_nqp_l{L}(int E, const NqpParams &p, hipStream_t s) {{
    switch (E) {{
{cases}
    default: return hipErrorInvalidValue;
    }}
}}

}}  // namespace nmfi
"""

_BATCH = """// Batched solve-kernel instantiations with {L} lane(s) per column
// (nqp_kernel.h).  Written by variants.py.
#include "nqp_kernel.h"

namespace nmfi {{

hipError_t launch_bnqp_l{L}(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,
                          int unit, hipStream_t s) {{
    switch (E) {{
{cases}
    default: return hipErrorInvalidValue;
    }}
}}

}}  // namespace nmfi
"""

_HEADER = """// Compiled solve-kernel variants (entries per lane E for each lanes-per-
// column L).  Written by variants.py.
#pragma once

#include <hip/hip_runtime.h>

namespace nmfi {{

struct NqpParams;
struct BSolveChunk;
struct BSolveProb;

{tables}

// E values compiled for L lanes per column (nullptr if none); *n = count.
inline const int *nqp_e_table(int L, int *n) {{
    switch (L) {{
{switch}
    default: *n = 0; return nullptr;
    }}
}}

{decls}

}}  // namespace nmfi
"""


def _write(path: str, text: str) -> None:
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


def generate() -> None:
    for L, es in VARIANTS.items():
        cases = "\n".join(f"    case {e}: return launch_nqp_t<{e}, {L}>(p, s);" for e in es)
        _write(os.path.join(CSRC, f"k_nqp_l{L}.hip"), _SOLO.format(L=L, cases=cases))
        cases = "\n".join(
            f"    case {e}: return launch_bnqp_t<{e}, {L}>(chunks, nchunks, queue, probs, max_inner, "
            f"eps, ls_guard, unit, s);" for e in es)
        _write(os.path.join(CSRC, f"k_nqp_b{L}.hip"), _BATCH.format(L=L, cases=cases))
    tables = "\n".join(
        f"constexpr int kNqpE{L}[] = {{{', '.join(str(e) for e in es)}}};" for L, es in VARIANTS.items())
    switch = "\n".join(
        f"    case {L}: *n = (int)(sizeof kNqpE{L} / sizeof(int)); return kNqpE{L};"
        for L in VARIANTS)
    decls = "\n".join(
        f"hipError_t launch_nqp_l{L}(int E, const NqpParams &p, hipStream_t s);\n"
        f"hipError_t launch_bnqp_l{L}(int E, const BSolveChunk *chunks, int nchunks, unsigned int *queue,\n"
        f"                          const BSolveProb *probs, int max_inner, double eps, int ls_guard,\n"
        f"                          int unit, hipStream_t s);" for L in VARIANTS)
    _write(os.path.join(CSRC, "nqp_variants.h"),
           _HEADER.format(tables=tables, switch=switch, decls=decls))


if __name__ == "__main__":
    generate()
