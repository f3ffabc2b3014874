"""Static check of the library's gfx950 assembly: no workgroup barrier
(s_barrier) inside a loop whose latch is exec-masked.

A loop whose exit the compiler takes as divergent is lowered with an exec
mask: lanes that leave wait outside the loop while the others go round again.
A barrier inside such a loop can then be passed by a wave with only some of
its lanes active, out of step with what the source says: in a work-queue loop
this lets threads run ahead of the thread that claims the next item (they
re-run a stale item and never finish).  Code whose barriers sit only in loops
with uniform (scalar-branch) latches is free of this.

The assembly's loop annotations name each block's innermost loop header
("in Loop: Header=BBx_y") and each header's nested loops ("Child Loop"); a
loop is exec-masked when one of its own blocks holds the lowering's
"s_andn2_b64 exec, exec, ..." step."""
import re


def parse(text):
    """Per function: its blocks (name, innermost loop header, instructions)
    and, per loop header, the headers of the loops nested in it."""
    funcs = {}
    cur = blk = None
    for line in text.splitlines():
        m = re.match(r"^([A-Za-z_$][\w$.]*):\s*(;.*)?$", line)
        if m and not line.startswith(".L"):
            cur = funcs.setdefault(m.group(1), {"blocks": [], "nested": {}})
            blk = {"name": "entry", "loop": None, "ins": []}
            cur["blocks"].append(blk)
            continue
        if cur is None:
            continue
        if line.startswith(".Lfunc_end"):
            cur = blk = None
            continue
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):\s*(;.*)?$", line)
        if m:
            name = m.group(1).replace(".L", "").replace("; %", "")
            com = m.group(2) or ""
            h = re.search(r"Header=(BB\d+_\d+) Depth=\d+", com)
            loop = name if "Loop Header" in com else (h.group(1) if h else None)
            blk = {"name": name, "loop": loop, "ins": []}
            cur["blocks"].append(blk)
            continue
        if re.match(r"^\s*;.*This (Inner )?Loop Header: Depth=\d+", line):
            blk["loop"] = blk["name"]
            continue
        m = re.match(r"^\s*;\s*Child Loop (BB\d+_\d+) Depth \d+", line)
        if m:
            cur["nested"].setdefault(blk["loop"], set()).add(m.group(1))
            continue
        s = line.strip()
        if s and not s.startswith((";", ".")):
            blk["ins"].append(s)
    return funcs


def barriers_in_masked_loops(funcs):
    """(function, loop header, barriers in the loop) for every exec-masked loop
    that holds a barrier, itself or in a nested loop."""
    bad = []
    for fn, f in funcs.items():
        loops = {b["loop"] for b in f["blocks"] if b["loop"]}
        for hdr in sorted(loops):
            inner = f["nested"].get(hdr, set())
            own = [b for b in f["blocks"] if b["loop"] == hdr]
            masked = any(i.startswith("s_andn2_b64 exec, exec,") for b in own for i in b["ins"])
            nbar = sum(i.startswith("s_barrier") for b in f["blocks"] if b["loop"] == hdr or b["loop"] in inner
                       for i in b["ins"])
            if masked and nbar:
                bad.append((fn, hdr, nbar))
    return bad


def barrier_count(funcs, name_part):
    return sum(i.startswith("s_barrier") for fn, f in funcs.items() if name_part in fn
               for b in f["blocks"] for i in b["ins"])
