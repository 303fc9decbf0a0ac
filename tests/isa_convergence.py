"""Static check of gfx950 kernel assembly: cross-lane reads under full exec.

The wave-per-order kernels exchange values between lanes (readlane,
readfirstlane, DPP, ds_bpermute/swizzle) on the assumption that all 64 lanes
are active there.  The compiler keeps that assumption only where control flow
reconverges the way the source suggests; where it does not (a lane-dependent
branch threaded around another one, for example), the wave reaches a
collective with some lanes masked off and reads stale registers of the masked
lanes.  This module parses the assembly text that hipcc emits, builds each
kernel's control-flow graph and runs a small dataflow analysis of the EXEC
mask:

  * exec is FULL at kernel entry (workgroups are whole waves);
  * s_and_saveexec / s_andn2_saveexec / writes of exec make it PARTIAL;
  * an SGPR pair that saved exec (or holds the complementary lanes of an
    if/else, or accumulates the lanes leaving a divergent loop) remembers the
    exec state that OR-ing it back restores;
  * at control-flow joins PARTIAL wins and disagreeing saved masks are lost.

A cross-lane instruction reached with exec possibly PARTIAL is reported,
except a readfirstlane of a value that the same block computed from scalar
operands with lane-independent arithmetic (every active lane holds it).
Readlane of the VGPRs that hold SGPR spills is exempt (spill code is
independent of exec), as are writelanes; a saved mask that is spilled to a VGPR
lane and reloaded keeps what it restores.
"""

from __future__ import annotations

import re
from dataclasses import dataclass, field

FULL, PARTIAL = "full", "partial"

_LABEL = re.compile(r"^(\.LBB\d+_\d+):")
_FUNC = re.compile(r"^([A-Za-z_$][\w.$]*):")
_SPILL = re.compile(r"\$vgpr(\d+) : SGPR spill to VGPR lane")
_DPP = ("quad_perm:", "row_shl:", "row_shr:", "row_ror:", "wave_shl", "wave_rol", "wave_shr",
        "wave_ror", "row_mirror", "row_half_mirror", "row_bcast", "row_newbcast")
_XLANE = ("v_readlane_b32", "v_readfirstlane_b32", "ds_bpermute_b32", "ds_permute_b32",
          "ds_swizzle_b32", "v_permlane16_swap_b32", "v_permlane32_swap_b32")
_NO_SDST = ("s_cmp", "s_bitcmp", "s_cbranch", "s_branch", "s_waitcnt", "s_nop", "s_setprio",
            "s_barrier", "s_sendmsg", "s_endpgm", "s_dcache", "s_sleep", "s_trap", "s_icache",
            "s_setpc", "s_set_gpr_idx")


def _sregs(op: str):
    """SGPR numbers named by one operand (sN or s[a:b]); vcc is 106/107."""
    m = re.fullmatch(r"s\[(\d+):(\d+)\]", op)
    if m:
        return list(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"s(\d+)", op)
    if m:
        return [int(m.group(1))]
    if op in ("vcc", "vcc_lo", "vcc_hi"):
        return [106, 107] if op == "vcc" else [106 if op == "vcc_lo" else 107]
    return []


def _pair(op: str):
    r = _sregs(op)
    return r[0] if len(r) == 2 else None


@dataclass
class Inst:
    line: int
    text: str
    mnem: str
    ops: list


@dataclass
class Block:
    name: str
    insts: list = field(default_factory=list)
    succ: list = field(default_factory=list)


@dataclass
class Function:
    name: str
    blocks: list
    spill_vgprs: set


def parse(asm: str):
    """Split assembly text into functions made of basic blocks."""
    funcs = []
    cur = None
    spill = set()
    blocks = []
    blk = None
    lines = asm.splitlines()

    def new_block(name):
        nonlocal blk
        blk = Block(name)
        blocks.append(blk)

    for no, raw in enumerate(lines, 1):
        line = raw.split(";")[0].rstrip() if not raw.lstrip().startswith(";") else ""
        sm = _SPILL.search(raw)
        if sm and cur is not None:
            spill.add(int(sm.group(1)))
        if not line.strip():
            continue
        if cur is None:
            fm = _FUNC.match(line)
            if fm and not line.startswith(".") and not line.startswith("__hip"):
                cur = fm.group(1)
                blocks, spill = [], set()
                new_block(cur)
            continue
        if line.startswith(".Lfunc_end"):
            funcs.append(Function(cur, blocks, spill))
            cur = None
            continue
        lm = _LABEL.match(line)
        if lm:
            if blk.insts or blk.name != cur:
                new_block(lm.group(1))
            else:
                new_block(lm.group(1))
            continue
        s = line.strip()
        if s.startswith("."):
            continue
        parts = s.split(None, 1)
        mnem = parts[0]
        ops = [o.strip() for o in parts[1].split(",")] if len(parts) > 1 else []
        blk.insts.append(Inst(no, s, mnem, ops))
        if mnem in ("s_endpgm", "s_branch") or mnem.startswith("s_cbranch") or mnem == "s_setpc_b64":
            new_block(f"{blk.name}+{no}")
    # successors
    for f in funcs:
        names = {b.name: i for i, b in enumerate(f.blocks)}
        for i, b in enumerate(f.blocks):
            last = b.insts[-1] if b.insts else None
            nxt = [f.blocks[i + 1].name] if i + 1 < len(f.blocks) else []
            if last is None:
                b.succ = nxt
            elif last.mnem == "s_endpgm" or last.mnem == "s_setpc_b64":
                b.succ = []
            elif last.mnem == "s_branch":
                b.succ = [last.ops[0]]
            elif last.mnem.startswith("s_cbranch"):
                b.succ = [last.ops[0]] + nxt
            else:
                b.succ = nxt
            for s in b.succ:
                if s not in names:
                    raise ValueError(f"{f.name}: branch to unknown label {s}")
    return funcs


def _drop(tok: dict, regs):
    for r in regs:
        tok.pop(r, None)
        tok.pop(r - 1, None)
        tok.pop(("half", r), None)


def _lane_operand(op: str):
    try:
        return int(op, 0)
    except ValueError:
        return None


def _spill_transfer(inst: Inst, tok: dict) -> bool:
    """SGPR spills to VGPR lanes: a saved exec mask spilled with writelane and
    reloaded with readlane keeps its token.  Returns True if handled."""
    m, ops = inst.mnem, inst.ops
    if m not in ("v_writelane_b32", "v_readlane_b32") or len(ops) != 3:
        return False
    lane = _lane_operand(ops[2])
    if m == "v_writelane_b32":
        v = re.fullmatch(r"v(\d+)", ops[0])
        src = _sregs(ops[1])
        if not v or lane is None:
            return True
        key = ("spill", int(v.group(1)), lane)
        t = None
        if len(src) == 1:
            r = src[0]
            if r in tok:
                t = (tok[r], 0)
            elif (r - 1) in tok:
                t = (tok[r - 1], 1)
        if t:
            tok[key] = t
        else:
            tok.pop(key, None)
        return True
    dst = _sregs(ops[0])
    v = re.fullmatch(r"v(\d+)", ops[1])
    _drop(tok, dst)
    if len(dst) != 1 or not v or lane is None:
        return True
    d = dst[0]
    slot = tok.get(("spill", int(v.group(1)), lane))
    if not slot:
        return True
    tok[("half", d)] = slot
    lo = d if slot[1] == 0 else d - 1
    a, b = tok.get(("half", lo)), tok.get(("half", lo + 1))
    if a and b and a[0] == b[0] and a[1] == 0 and b[1] == 1:
        tok[lo] = a[0]
    return True


def _transfer(inst: Inst, exec_state: str, tok: dict):
    """Apply one instruction to (exec, tokens); returns the new exec state.

    tok maps the low register of an SGPR pair to (kind, R):
      ("save", R)  OR-ing it into exec restores exec state R (a mask saved
                   by saveexec, the complementary lanes of an if/else, or an
                   accumulator of lanes that left a divergent loop);
      ("copy", R)  a copy of exec taken in state R;
      ("sub", R)   a subset of such a copy (copy AND condition).
    """
    m, ops = inst.mnem, inst.ops
    if m.endswith("saveexec_b64") and ops:
        d = _pair(ops[0])
        src = _pair(ops[1]) if len(ops) > 1 else None
        new_exec = PARTIAL
        if m == "s_and_saveexec_b64":
            new_tok = ("save", exec_state)
        elif m == "s_andn2_saveexec_b64" and tok.get(src, ("", None))[0] == "save":
            # exec = S & ~exec, D = old exec: D and the new exec partition what S restored
            new_tok = ("save", tok[src][1])
        elif m == "s_or_saveexec_b64" and tok.get(src, ("", None))[0] == "save":
            # the else entry of an if/else: S holds the lanes that the then-block
            # (the current exec) lacks, so exec | S is the state S restores, and
            # D = the then-lanes restore it again after the else-block
            new_tok = ("save", tok[src][1])
            new_exec = tok[src][1]
        else:
            new_tok = None
        if d is not None:
            _drop(tok, (d, d + 1))
            if new_tok:
                tok[d] = new_tok
        return new_exec
    if ops and ops[0] == "exec":
        if m == "s_or_b64" and len(ops) == 3 and "exec" in ops[1:]:
            other = ops[2] if ops[1] == "exec" else ops[1]
            t = tok.get(_pair(other))
            # OR-ing back a saved mask, or a copy of the whole exec, restores it
            if t and t[0] in ("save", "copy") and t[1] == FULL:
                return FULL
            return exec_state if exec_state == FULL else PARTIAL
        if m == "s_mov_b64" and len(ops) == 2:
            t = tok.get(_pair(ops[1]))
            return FULL if (t and t[0] == "copy" and t[1] == FULL) else PARTIAL
        return PARTIAL
    if m.startswith("s_") and ops and not m.startswith(_NO_SDST):
        d = _pair(ops[0])
        keep = None
        srcs = ops[1:]
        tks = [tok.get(_pair(o)) if o != "exec" else ("exec", exec_state) for o in srcs]
        kinds = [t[0] if t else None for t in tks]
        if m == "s_mov_b64" and d is not None and len(srcs) == 1:
            if srcs[0] == "exec":
                keep = ("copy", exec_state)
            elif srcs[0] in ("0", "0x0"):
                keep = ("save", exec_state)
            elif tks[0] and kinds[0] != "exec":
                keep = tks[0]
        elif m == "s_or_b64" and d is not None and len(srcs) == 2 and ops[0] in srcs and \
                tok.get(d, ("", None))[0] == "save":
            keep = tok[d]
        elif m == "s_xor_b64" and d is not None and len(srcs) == 2:
            if "exec" in kinds:
                other = tks[1 - kinds.index("exec")]
                if other and other[0] == "save":
                    keep = other
            elif sorted(k or "" for k in kinds) == ["copy", "sub"]:
                # copy ^ (copy & cond): the lanes of the copy outside the subset
                keep = ("save", tks[kinds.index("copy")][1])
        elif m == "s_and_b64" and d is not None and len(srcs) == 2 and "copy" in kinds:
            keep = ("sub", tks[kinds.index("copy")][1])
        _drop(tok, _sregs(ops[0]))
        if keep is not None and d is not None:
            tok[d] = keep
        return exec_state
    if _spill_transfer(inst, tok):
        return exec_state
    if m.startswith("v_") or m.startswith("s_load") or m.startswith("s_buffer_load"):
        for op in ops:
            regs = _sregs(op)
            if regs and (op is ops[0] or "_co_" in m or m.startswith("v_cmp") or m.startswith("v_div_scale")):
                _drop(tok, regs)
    return exec_state


def _is_xlane(inst: Inst, spill: set) -> bool:
    if inst.mnem in _XLANE:
        if inst.mnem == "v_readlane_b32" and len(inst.ops) > 1:
            m = re.fullmatch(r"v(\d+)", inst.ops[1])
            if m and int(m.group(1)) in spill:
                return False
        return True
    return any(d in inst.text for d in _DPP)


# VALU operations whose result depends only on their operands (no lane mask,
# lane id or cross-lane read): with only scalar operands, every active lane
# computes the same value.
_UNIFORM_VALU = ("v_add_u32", "v_add_co_u32", "v_sub_u32", "v_sub_co_u32", "v_subrev_u32",
                 "v_subrev_co_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_lshlrev_b32", "v_lshlrev_b64",
                 "v_lshrrev_b32", "v_lshrrev_b64", "v_ashrrev_i32", "v_and_b32", "v_or_b32", "v_xor_b32",
                 "v_mov_b32", "v_mov_b64", "v_bfe_u32", "v_min_u32", "v_max_u32", "v_not_b32", "v_add3_u32")


def _scalar_operand(op: str) -> bool:
    return bool(re.fullmatch(r"s\d+|s\[\d+:\d+\]|-?\d+|0x[0-9a-fA-F]+", op))


def _uniform_source(insts, k: int) -> bool:
    """A readfirstlane at insts[k] whose source VGPR was last written, in the
    same block, by a lane-independent VALU operation on scalar operands only:
    all active lanes hold the same value, so reading the first one is exact."""
    src = insts[k].ops[1] if len(insts[k].ops) > 1 else ""
    m = re.fullmatch(r"v(\d+)", src)
    if not m:
        return False
    reg = int(m.group(1))
    for inst in reversed(insts[:k]):
        if not inst.ops:
            continue
        d = inst.ops[0]
        md = re.fullmatch(r"v(\d+)|v\[(\d+):(\d+)\]", d)
        if not md:
            continue
        lo, hi = (int(md.group(1)),) * 2 if md.group(1) else (int(md.group(2)), int(md.group(3)))
        if not lo <= reg <= hi:
            continue
        base = re.sub(r"_e(32|64)$", "", inst.mnem)
        if base not in _UNIFORM_VALU:
            return False
        srcs = inst.ops[1:]
        if "_co_" in base and srcs:
            srcs = srcs[1:]  # the carry-out mask is a destination
        return all(_scalar_operand(o) for o in srcs)
    return False


def _merge(a, b):
    if a is None:
        return b
    ea, ta = a
    eb, tb = b
    e = FULL if (ea == FULL and eb == FULL) else PARTIAL
    t = {k: v for k, v in ta.items() if k in tb and tb[k] == v}
    return e, t


def analyse(func: Function):
    """Returns (cross-lane instructions under possibly partial exec, divergent loop exits)."""
    idx = {b.name: i for i, b in enumerate(func.blocks)}
    state_in = [None] * len(func.blocks)
    state_in[0] = (FULL, {})
    work = [0]
    while work:
        i = work.pop()
        e, t = state_in[i]
        t = dict(t)
        for inst in func.blocks[i].insts:
            e = _transfer(inst, e, t)
        for s in func.blocks[i].succ:
            j = idx[s]
            new = _merge(state_in[j], (e, t))
            if new != state_in[j]:
                state_in[j] = new
                work.append(j)
    bad = []
    div_loops = 0
    for i, b in enumerate(func.blocks):
        if state_in[i] is None:
            continue
        e, t = state_in[i]
        t = dict(t)
        for k, inst in enumerate(b.insts):
            if inst.mnem == "s_andn2_b64" and inst.ops[:2] == ["exec", "exec"]:
                div_loops += 1
            if e != FULL and _is_xlane(inst, func.spill_vgprs):
                if not (inst.mnem == "v_readfirstlane_b32" and _uniform_source(b.insts, k)):
                    bad.append((inst.line, inst.text))
            e = _transfer(inst, e, t)
    return bad, div_loops


def check(asm: str):
    """{function name: (bad cross-lane instructions, divergent loop exits)}."""
    return {f.name: analyse(f) for f in parse(asm)}
