"""Source instrumentation of HIP kernels for the race checker.

The paper instruments CUDA kernels with a source-to-source rewriter built on
Clang (Sec. IV-A): every access to monitored shared or global data gets a
call of the shadow update, and every barrier becomes a barrier that also
advances the thread's clocks.  This module does the same for HIP: it reads
the kernel's syntax tree from ROCm's clang (``-ast-dump=json``), finds the
array accesses and barriers, and rewrites the source text:

* ``p[i]`` on a pointer parameter ``p`` (global memory) becomes
  ``(*hr_gat<K>(hr_a, hr_m, hr_t, slot, p, (i), line))``, which checks the
  access and returns the element's address, so reads, writes, compound
  assignments, increments and ``atomicXxx(&p[i], ...)`` keep their meaning;
* ``s[i]`` on a ``__shared__`` array ``s`` (LDS) becomes
  ``(*hr_lat<K>(hr_a.env, hr_t, hr_sh_s, N, id, s, (i), line))`` with an LDS
  shadow array ``hr_sh_s`` cleared at kernel start;
* ``__syncthreads()`` becomes ``hr_barrier_block(hr_a.env, hr_t)``, and
  ``__syncwarp(mask)`` becomes ``hr_barrier_mask(hr_a.env, hr_t, mask)``
  (``__syncwarp()``: the full mask), which takes the barrier at the level
  the mask names for the calling lane: its whole wave, or its whole aligned
  tile of the context's tile width (``hr_config.wave_bits``), which HIP
  code reaches by letting each tile call ``__syncwarp`` with its own lanes'
  mask.  A mask narrower than that orders nothing for the checker, and the
  report warns of it.

K is the access kind decided from the expression around the subscript: the
left side of ``=`` is a write, of a compound assignment or ``++``/``--`` a read
and a write, the operand of ``&`` passed to an atomic function an atomic, and
an lvalue-to-rvalue conversion a read.  The call-site id of each hook is the
source line.  Subscripts of other shapes (multi-dimensional arrays, members,
an address taken for another use, elements not 4 bytes wide) are left
unchecked and listed in the report.

Each kernel becomes a template over the checker's thread state
(``hr_thread``: block and wave, or tile, barriers; ``hr_tn``: tiles nested
in waves, for a context made with ``HR_CFG_NESTED_TILES``), gains two
parameters (``hr_kargs hr_a, hr_rmap hr_m``) and an ``extern "C"`` launcher ``hr_launch_<kernel>(ctx, regions, n_regions, grid,
block, lds_bytes, stream, <original parameters>)``; ``regions[j]`` is the
context region (from ``hr_shadow_alloc``) of the kernel's j-th pointer
parameter, which must point at the region's start.  The launcher runs the
instance the context asks for.  Kernels that are already templates, or that
have C linkage, are not supported.
"""
from __future__ import annotations

import dataclasses
import json
import os
import re
import subprocess
import sys
from typing import Dict, List, Optional, Tuple

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)

ATOMICS = {"atomicAdd", "atomicSub", "atomicExch", "atomicMin", "atomicMax", "atomicInc",
           "atomicDec", "atomicCAS", "atomicAnd", "atomicOr", "atomicXor"}
WORD_TYPES = {"float", "int", "unsigned int", "unsigned", "int32_t", "uint32_t"}
KIND = {"R": 0, "W": 1, "A": 2, "RW": 3}


def clang() -> str:
    for cand in (os.environ.get("HR_CLANG"), "/opt/rocm/llvm/bin/clang++"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("ROCm clang++ not found")


def _decode_all(text: str) -> list:
    dec, i, out = json.JSONDecoder(), 0, []
    while True:
        while i < len(text) and text[i].isspace():
            i += 1
        if i >= len(text):
            return out
        obj, i = dec.raw_decode(text, i)
        out.append(obj)


def kernel_names(src: str) -> List[str]:
    """Names of __global__ functions, read from the source text."""
    return re.findall(r"__global__\s+(?:__launch_bounds__\s*\([^)]*\)\s*)?void\s+(\w+)\s*\(", src)


def dump_kernel(path: str, name: str, extra_args=()) -> Optional[dict]:
    """The FunctionDecl of kernel `name` defined in `path`, as clang's JSON."""
    cmd = [clang(), "-x", "hip", "--offload-arch=gfx950", "--cuda-device-only", "-fsyntax-only",
           "-Xclang", "-ast-dump=json", "-Xclang", f"-ast-dump-filter={name}",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), *extra_args, path]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"clang failed on {path}:\n{res.stderr}")
    for node in _decode_all(res.stdout):
        if node.get("kind") != "FunctionDecl" or node.get("name") != name:
            continue
        if not any(c.get("kind") == "CompoundStmt" for c in node.get("inner", [])):
            continue                              # a declaration, not the definition
        if any(c.get("kind") == "CUDAGlobalAttr" for c in node.get("inner", [])):
            return node
    return None


def _off(loc: dict) -> Optional[int]:
    if "offset" in loc:
        return loc["offset"]
    if "expansionLoc" in loc:
        return loc["expansionLoc"].get("offset")
    return None


def _tok(loc: dict) -> int:
    if "tokLen" in loc:
        return loc["tokLen"]
    return loc.get("expansionLoc", {}).get("tokLen", 0)


def span(node: dict) -> Tuple[int, int]:
    r = node["range"]
    b, e = _off(r["begin"]), _off(r["end"])
    return b, e + _tok(r["end"])


def _strip(node: dict) -> dict:
    while node.get("kind") in ("ImplicitCastExpr", "ParenExpr") and node.get("inner"):
        node = node["inner"][0]
    return node


@dataclasses.dataclass
class Edit:
    start: int
    end: int
    kind: str                 # 'g' global subscript, 'l' LDS subscript, 'bar' barrier
    parts: Tuple = ()         # (prefix, (index start, index end), suffix) for subscripts


@dataclasses.dataclass
class Report:
    kernel: str
    global_sites: int = 0
    lds_sites: int = 0
    barriers: int = 0
    skipped: List[str] = dataclasses.field(default_factory=list)
    pointer_params: List[str] = dataclasses.field(default_factory=list)
    shared_arrays: List[Tuple[str, int]] = dataclasses.field(default_factory=list)


def _line_of(src: str, off: int) -> int:
    return src.count("\n", 0, off) + 1


def _callee(call: dict) -> str:
    inner = call.get("inner") or []
    if not inner:
        return ""
    d = _strip(inner[0])
    return (d.get("referencedDecl") or {}).get("name", "") if d.get("kind") == "DeclRefExpr" else ""


def _transparent(node: dict, child: dict) -> bool:
    """Parents that pass an lvalue through unchanged: parentheses, no-op
    casts, and the value operands of a conditional operator."""
    k = node.get("kind")
    if k == "ParenExpr":
        return True
    if k == "ImplicitCastExpr" and node.get("castKind") == "NoOp":
        return True
    if k == "ConditionalOperator":
        return (node.get("inner") or [None])[0] is not child
    return False


def _kind_of(sub: dict, parents: List[dict]) -> Optional[str]:
    j = len(parents) - 1
    while j >= 0 and _transparent(parents[j], parents[j + 1] if j + 1 < len(parents) else sub):
        sub = parents[j]
        j -= 1
    p = parents[j] if j >= 0 else {}
    g = parents[j - 1] if j >= 1 else {}
    pk = p.get("kind")
    first = (p.get("inner") or [None])[0] is sub
    if pk == "BinaryOperator" and p.get("opcode") == "=" and first:
        return "W"
    if pk == "CompoundAssignOperator" and first:
        return "RW"
    if pk == "UnaryOperator" and p.get("opcode") in ("++", "--"):
        return "RW"
    if pk == "UnaryOperator" and p.get("opcode") == "&":
        return "A" if g.get("kind") == "CallExpr" and _callee(g) in ATOMICS else None
    if pk == "ImplicitCastExpr" and p.get("castKind") == "LValueToRValue":
        return "R"
    return None


def analyse(src: str, fn: dict) -> Tuple[List[Edit], Report, dict]:
    """Edits for one kernel, its report, and positions for the signature and
    prologue."""
    rep = Report(fn["name"])
    params = [c for c in fn.get("inner", []) if c.get("kind") == "ParmVarDecl"]
    body = next(c for c in fn["inner"] if c.get("kind") == "CompoundStmt")
    slot: Dict[str, int] = {}
    for p in params:
        if p.get("type", {}).get("qualType", "").rstrip().endswith("*"):
            slot[p["id"]] = len(rep.pointer_params)
            rep.pointer_params.append(p["name"])
    shared: Dict[str, Tuple[int, str, int]] = {}     # decl id -> (array id, name, words)
    edits: List[Edit] = []

    def visit(node: dict, parents: List[dict]):
        k = node.get("kind")
        if k == "VarDecl" and any(c.get("kind") == "CUDASharedAttr" for c in node.get("inner", [])):
            m = re.fullmatch(r"(?:volatile\s+)?([\w ]+?)\s*\[(\d+)\]", node["type"]["qualType"])
            if m and m.group(1).strip() in WORD_TYPES:
                shared[node["id"]] = (len(shared), node["name"], int(m.group(2)))
                rep.shared_arrays.append((node["name"], int(m.group(2))))
            else:
                rep.skipped.append(f"shared {node['name']}: {node['type']['qualType']}")
        if k == "CallExpr" and _callee(node) == "__syncthreads":
            b, e = span(node)
            edits.append(Edit(b, e, "bar"))
            rep.barriers += 1
        if k in ("CallExpr", "CXXMemberCallExpr"):
            _cg_sync(src, node, edits, rep)
        if k == "CallExpr" and _callee(node) == "__syncwarp":
            b, e = span(node)
            args = (node.get("inner") or [])[1:]
            if args:                            # the mask expression, itself rewritten
                edits.append(Edit(b, e, "wbar", ("hr_barrier_mask(hr_a.env, hr_t, "
                                                 "(unsigned long long)(", span(args[0]), "))")))
            else:
                edits.append(Edit(b, e, "wbar"))
            rep.barriers += 1
        if k == "ArraySubscriptExpr":
            base = _strip(node["inner"][0])
            ref = base.get("referencedDecl") or {}
            line = _line_of(src, span(node)[0])
            where = None
            if base.get("kind") == "DeclRefExpr" and ref.get("id") in slot:
                where = "g"
            elif base.get("kind") == "DeclRefExpr" and ref.get("id") in shared:
                where = "l"
            if where:
                kind = _kind_of(node, parents)
                ty = node.get("type", {}).get("qualType", "")
                ty = re.sub(r"\b(const|volatile)\b", "", ty).strip()
                if kind is None:
                    rep.skipped.append(f"line {line}: {ref.get('name')}[...] in an unsupported context")
                elif ty not in WORD_TYPES:
                    rep.skipped.append(f"line {line}: {ref.get('name')}[...] of type {ty}")
                else:
                    b, e = span(node)
                    ib, ie = span(node["inner"][1])
                    name = ref["name"]
                    if where == "g":
                        pre = (f"(*hr_gat<{KIND[kind]}>(hr_a, hr_m, hr_t, {slot[ref['id']]}, "
                               f"{name}, (")
                        rep.global_sites += 1
                    else:
                        aid, _, words = shared[ref["id"]]
                        pre = (f"(*hr_lat<{KIND[kind]}>(hr_a.env, hr_t, hr_sh_{name}, {words}, "
                               f"{aid}, {name}, (")
                        rep.lds_sites += 1
                    edits.append(Edit(b, e, where, (pre, (ib, ie), f"), {line}))")))
        for c in node.get("inner", []) or []:
            visit(c, parents + [node])

    visit(body, [fn])
    last = params[-1] if params else None
    pos = {"params_end": span(last)[1] if last else None,
           "body_open": span(body)[0],
           "params": [(p["name"], src[span(p)[0]:span(p)[1]]) for p in params]}
    return edits, rep, pos


def _cg_sync(src: str, node: dict, edits: List[Edit], rep: Report) -> bool:
    """A cooperative-groups sync(): on a thread_block_tile<N> it becomes the
    checker's barrier for the calling lane's aligned N-lane tile (its wave
    when N is 64), on a thread_block the block barrier.  Other groups (grid,
    coalesced and run-time sized groups) are left as they are and reported:
    the checker then orders nothing there, which may report more races,
    never fewer."""
    inner = node.get("inner") or []
    if not inner:
        return False
    callee = _strip(inner[0])
    if callee.get("kind") != "MemberExpr" or callee.get("name") != "sync":
        return False
    base = _strip((callee.get("inner") or [{}])[0])
    ty = base.get("type", {})
    text = " ".join(t for t in (ty.get("qualType", ""), ty.get("desugaredQualType", "")) if t)
    b, e = span(node)
    m = re.search(r"thread_block_tile<\s*(\d+)", text)
    if m:
        n = int(m.group(1))
        edits.append(Edit(b, e, "text", (f"hr_barrier_mask(hr_a.env, hr_t, hr_lane_tile_mask({n}))",)))
        rep.barriers += 1
        return True
    if re.search(r"(^|[\s:])thread_block\b", text):
        edits.append(Edit(b, e, "bar"))
        rep.barriers += 1
        return True
    if "cooperative_groups" in text or re.search(r"(grid|coalesced|thread)_group", text):
        rep.skipped.append(f"line {_line_of(src, b)}: sync() of {text.split()[0]} is not modelled")
    return False


def _apply(src: str, lo: int, hi: int, edits: List[Edit]) -> str:
    """src[lo:hi] with the edits inside that range applied (nested edits
    inside a subscript's index are applied recursively)."""
    inside = sorted((e for e in edits if lo <= e.start and e.end <= hi), key=lambda e: (e.start, -e.end))
    out, cur = [], lo
    i = 0
    while i < len(inside):
        e = inside[i]
        if e.start < cur:                       # nested in an edit already applied
            i += 1
            continue
        out.append(src[cur:e.start])
        if e.kind == "bar":
            out.append("hr_barrier_block(hr_a.env, hr_t)")
        elif e.kind == "wbar" and not e.parts:
            out.append("hr_barrier_mask(hr_a.env, hr_t, ~0ull)")
        elif e.kind == "text":
            out.append(e.parts[0])
        else:
            pre, (ib, ie), post = e.parts
            nested = [x for x in edits if ib <= x.start and x.end <= ie and x is not e]
            out.append(pre + _apply(src, ib, ie, nested) + post)
        cur = e.end
        i += 1
    out.append(src[cur:hi])
    return "".join(out)


def _launcher(name: str, rep: Report, params: List[Tuple[str, str]]) -> str:
    decl = ", ".join(text for _, text in params)
    args = ", ".join(n for n, _ in params)
    sep = ", " if params else ""
    n = len(rep.pointer_params)
    return f"""
extern "C" hr_status hr_launch_{name}(hr_ctx hr_c, const uint32_t* hr_regions,
                                     uint32_t hr_n_regions, unsigned hr_gx, unsigned hr_gy,
                                     unsigned hr_gz, unsigned hr_bx, unsigned hr_by, unsigned hr_bz,
                                     size_t hr_lds, void* hr_stream{sep}{decl})
{{
    if (hr_n_regions != {n}u || ({n}u && !hr_regions)) return HR_E_INVAL;
    hr_kargs hr_a;
    size_t hr_size = 0;
    if (hr_dev_args(hr_c, &hr_a, sizeof hr_a, &hr_size) != HR_OK || hr_size != sizeof hr_a)
        return HR_E_INVAL;
    hr_rmap hr_m = {{}};
    for (uint32_t j = 0; j < {n}u; ++j) {{
        if (hr_regions[j] >= HR_MAX_REGIONS) return HR_E_INVAL;
        hr_m.id[j] = hr_regions[j];
    }}
    (void)hipGetLastError();
    if (hr_a.env.nested)
        hipLaunchKernelGGL({name}<hr_tn>, dim3(hr_gx, hr_gy, hr_gz), dim3(hr_bx, hr_by, hr_bz),
                           hr_lds, (hipStream_t)hr_stream{sep}{args}, hr_a, hr_m);
    else
        hipLaunchKernelGGL({name}<hr_thread>, dim3(hr_gx, hr_gy, hr_gz),
                           dim3(hr_bx, hr_by, hr_bz), hr_lds, (hipStream_t)hr_stream{sep}{args},
                           hr_a, hr_m);
    return hipGetLastError() == hipSuccess ? HR_OK : HR_E_HIP;
}}
"""


def _template_point(src: str, name: str) -> int:
    """Where `template <class hr_T>` goes before kernel `name`'s definition:
    at the start of the line that holds its __global__ (so a leading
    `static` stays after it)."""
    ms = [m for m in re.finditer(r"__global__\s+(?:__launch_bounds__\s*\([^)]*\)\s*)?void\s+"
                                 + re.escape(name) + r"\s*\(", src)]
    if len(ms) != 1:
        raise RuntimeError(f"{name}: expected one definition, found {len(ms)}")
    line = src.rfind("\n", 0, ms[0].start()) + 1
    lead = src[line:ms[0].start()]
    if re.search(r"\btemplate\b|extern\s*\"C\"", src[max(0, line - 200):ms[0].start()]
                 .split(";")[-1].split("}")[-1]):
        raise RuntimeError(f"{name}: template kernels and kernels with C linkage are not supported")
    if lead.strip() and lead.strip() not in ("static", "inline", "static inline"):
        raise RuntimeError(f"{name}: unsupported declaration prefix {lead.strip()!r}")
    return line


def instrument(path: str, kernels: Optional[List[str]] = None, extra_args=()) -> Tuple[str, List[Report]]:
    """Instrumented source of the file at `path` and one report per kernel."""
    src = open(path).read()
    names = kernels or kernel_names(src)
    edits_all: List[Edit] = []
    inserts: List[Tuple[int, str]] = []
    reports, launchers = [], []
    for name in names:
        fn = dump_kernel(path, name, extra_args)
        if fn is None:
            raise RuntimeError(f"kernel {name} not found in {path}")
        edits, rep, pos = analyse(src, fn)
        if len(rep.pointer_params) > 8:
            raise RuntimeError(f"{name}: more than 8 pointer parameters")
        inserts.append((_template_point(src, name), "template <class hr_T>\n"))
        edits_all += edits
        sig = ", hr_kargs hr_a, hr_rmap hr_m" if pos["params_end"] is not None else \
              "hr_kargs hr_a, hr_rmap hr_m"
        if pos["params_end"] is not None:
            inserts.append((pos["params_end"], sig))
        else:                                   # no parameters: insert inside "()"
            inserts.append((src.index("(", src.index(name, span(fn)[0])) + 1, sig))
        pro = ["", "    hr_T hr_t = hr_start<hr_T>(hr_a.env, blockIdx.x + gridDim.x * "
                   "(blockIdx.y + gridDim.y * blockIdx.z), threadIdx.x + blockDim.x * "
                   "(threadIdx.y + blockDim.y * threadIdx.z));"]
        for arr, words in rep.shared_arrays:
            pro.append(f"    __shared__ uint32_t hr_sh_{arr}[{words}];")
        if rep.shared_arrays:
            pro.append("    for (uint32_t hr_i = hr_t.thread; hr_i < %d; "
                       "hr_i += blockDim.x * blockDim.y * blockDim.z) {"
                       % max(w for _, w in rep.shared_arrays))
            for arr, words in rep.shared_arrays:
                pro.append(f"        if (hr_i < {words}) hr_sh_{arr}[hr_i] = 0;")
            pro.append("    }")
            pro.append("    __syncthreads();   // LDS shadow cleared before any access")
        inserts.append((pos["body_open"] + 1, "\n".join(pro)))
        launchers.append(_launcher(name, rep, pos["params"]))
        reports.append(rep)
    # apply: edits (non-overlapping at top level) and insertions
    points = sorted(set([0, len(src)] + [p for p, _ in inserts]))
    out = [text for p, text in inserts if p == 0]
    for a, b in zip(points[:-1], points[1:]):
        out.append(_apply(src, a, b, edits_all))
        out.extend(text for p, text in inserts if p == b)
    body = "".join(out)
    head = ('// Instrumented by paper_2401_04701_amd.instrument: every checked access calls\n'
            '// the race checker\'s shadow update (hr_gat / hr_lat), barriers advance its\n'
            '// clocks.  Generated file.\n#include "hr_nested.h"\n')
    return head + body + "".join(launchers), reports


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="Instrument HIP kernels for the race checker")
    ap.add_argument("source")
    ap.add_argument("-o", "--output", required=True)
    ap.add_argument("-k", "--kernel", action="append", help="kernel name (default: all)")
    args = ap.parse_args(argv)
    text, reports = instrument(args.source, args.kernel)
    with open(args.output, "w") as f:
        f.write(text)
    for r in reports:
        print(f"{r.kernel}: {r.global_sites} global and {r.lds_sites} LDS access sites, "
              f"{r.barriers} barriers; regions {r.pointer_params}", file=sys.stderr)
        for s in r.skipped:
            print(f"  not checked: {s}", file=sys.stderr)


if __name__ == "__main__":
    main()
