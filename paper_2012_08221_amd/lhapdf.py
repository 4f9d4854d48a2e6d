"""Reader and writer for the community PDF grid format and folder structure
(the standard format agreed for PDF sets, Sec. 1; the same data folders are
read unchanged, Sec. 4).

A set called NAME is a folder NAME/ holding NAME.info (YAML metadata for the
whole set) and one file NAME_MMMM.dat per member (MMMM = member number, four
digits).  A member file is a YAML header followed by subgrid blocks, each
section ending with a line "---".  A block has one line of x knots, one line of
Q knots (GeV), one line of parton ids, then one line per (x, Q) knot pair with
the x f values of every parton in that order, Q running fastest.  Neighbouring
blocks repeat their common Q knot (a flavour threshold).

The reader turns one member into the library's grid description: the x knots
(every block must share them), the Q^2 knots of all blocks concatenated with
the repeated threshold knots kept, the block offsets, the values as
[parton][x][Q^2], and the alpha_s knots (AlphaS_Qs squared, AlphaS_Vals) from
the member header or else the set's info file.  Everything here is host-side
text handling; evaluation is done by the library's kernels.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np
import yaml

__all__ = ["MemberGrid", "FormatError", "read_member", "read_info", "find_set", "load_member",
           "load_set", "write_set", "parse_name"]


@dataclass
class MemberGrid:
    """One member in the library's layout (the fields a grid description needs)."""
    pids: np.ndarray                 # int32 [n_flav]
    x: np.ndarray                    # [n_x]
    q2: np.ndarray                   # [n_q], blocks concatenated, threshold knots repeated
    q_off: np.ndarray                # int32 [n_sub + 1]
    xf: np.ndarray                   # [n_flav][n_x][n_q]
    as_q2: np.ndarray = field(default_factory=lambda: np.zeros(0))
    as_val: np.ndarray = field(default_factory=lambda: np.zeros(0))
    meta: dict = field(default_factory=dict)   # header merged over the set's info


class FormatError(ValueError):
    pass


def _floats(line: str, what: str, path: str) -> np.ndarray:
    try:
        return np.array(line.split(), dtype=np.float64)
    except ValueError as e:
        raise FormatError("%s: bad %s line: %s" % (path, what, e)) from None


def _sections(text: str):
    """Split at lines that are exactly '---' (surrounding blanks ignored)."""
    out, cur = [], []
    for line in text.splitlines():
        if line.strip() == "---":
            out.append(cur)
            cur = []
        else:
            cur.append(line)
    if any(s.strip() for s in cur):
        out.append(cur)
    return out


def read_info(path: str) -> dict:
    """The set's metadata (NAME.info) as a dict."""
    with open(path) as fh:
        meta = yaml.safe_load(fh) or {}
    if not isinstance(meta, dict):
        raise FormatError("%s: metadata is not a mapping" % path)
    return meta


def read_member(path: str, info: dict | None = None) -> MemberGrid:
    """One member file (NAME_MMMM.dat) -> MemberGrid; info supplies the
    set-level metadata that the member header does not override."""
    with open(path) as fh:
        secs = _sections(fh.read())
    if len(secs) < 2:
        raise FormatError("%s: no subgrid block after the header" % path)
    header = yaml.safe_load("\n".join(secs[0])) or {}
    if not isinstance(header, dict):
        raise FormatError("%s: header is not a mapping" % path)
    meta = dict(info or {})
    meta.update(header)
    fmt = meta.get("Format", "lhagrid1")
    if fmt != "lhagrid1":
        raise FormatError("%s: format %r is not lhagrid1" % (path, fmt))

    x = None
    pids = None
    qs, blocks = [], []
    for b, sec in enumerate(secs[1:]):
        lines = [ln for ln in sec if ln.strip()]
        if not lines:
            continue
        if len(lines) < 3:
            raise FormatError("%s: block %d has no knot or parton lines" % (path, b))
        xb = _floats(lines[0], "x knot", path)
        qb = _floats(lines[1], "Q knot", path)
        try:
            pb = np.array([int(t) for t in lines[2].split()], dtype=np.int32)
        except ValueError:
            raise FormatError("%s: block %d: bad parton id line" % (path, b)) from None
        rows = lines[3:]
        if len(rows) != xb.size * qb.size:
            raise FormatError("%s: block %d has %d value lines, expected %d x %d"
                              % (path, b, len(rows), xb.size, qb.size))
        if any(len(r.split()) != pb.size for r in rows):
            raise FormatError("%s: block %d: every value line needs %d entries" % (path, b, pb.size))
        vals = _floats(" ".join(rows), "value", path).reshape(len(rows), pb.size)
        if x is None:
            x, pids = xb, pb
        else:
            if xb.shape != x.shape or np.any(xb != x):
                raise FormatError("%s: block %d has other x knots than block 0 (a shared x axis "
                                  "is required)" % (path, b))
            if pb.shape != pids.shape or np.any(pb != pids):
                raise FormatError("%s: block %d has another parton list" % (path, b))
        qs.append(qb)
        # file order: x outer, Q inner, partons across -> [parton][x][Q]
        blocks.append(vals.reshape(xb.size, qb.size, pb.size).transpose(2, 0, 1))
    if x is None:
        raise FormatError("%s: no subgrid block" % path)
    for s in range(1, len(qs)):
        if qs[s - 1][-1] != qs[s][0]:
            raise FormatError("%s: blocks %d and %d do not share their boundary Q knot"
                              % (path, s - 1, s))
    q_off = np.concatenate([[0], np.cumsum([q.size for q in qs])]).astype(np.int32)
    q = np.concatenate(qs)
    g = MemberGrid(pids=pids, x=x, q2=q * q, q_off=q_off,
                   xf=np.ascontiguousarray(np.concatenate(blocks, axis=2)), meta=meta)
    aq, av = meta.get("AlphaS_Qs"), meta.get("AlphaS_Vals")
    if aq is not None and av is not None:
        aq = np.asarray(aq, dtype=np.float64)
        av = np.asarray(av, dtype=np.float64)
        if aq.shape != av.shape:
            raise FormatError("%s: AlphaS_Qs and AlphaS_Vals differ in length" % path)
        g.as_q2, g.as_val = aq * aq, av
    return g


def parse_name(spec: str) -> tuple[str, int]:
    """'NAME/M' or 'NAME' (member 0) -> (NAME, M)."""
    name, _, mem = spec.partition("/")
    if not name:
        raise ValueError("empty set name in %r" % spec)
    return name, int(mem) if mem else 0


def find_set(name: str, dirname: str | None = None) -> str:
    """Folder of set NAME: under dirname if given, else the first entry of
    LHAPDF_DATA_PATH (colon-separated) that holds it."""
    env = os.environ.get("LHAPDF_DATA_PATH", "")
    roots = [dirname] if dirname else [p for p in env.split(":") if p]
    for r in roots:
        d = os.path.join(r, name)
        if os.path.isfile(os.path.join(d, name + ".info")) or os.path.isdir(d):
            return d
    raise FileNotFoundError("PDF set %r not found under %s"
                            % (name, roots or "LHAPDF_DATA_PATH (unset)"))


def load_member(spec: str, dirname: str | None = None) -> MemberGrid:
    """Member 'NAME/M' of a set (the paper's mkPDF naming, Fig. 1)."""
    name, mem = parse_name(spec)
    d = find_set(name, dirname)
    ipath = os.path.join(d, name + ".info")
    info = read_info(ipath) if os.path.isfile(ipath) else {}
    return read_member(os.path.join(d, "%s_%04d.dat" % (name, mem)), info)


def load_set(name: str, dirname: str | None = None) -> list[MemberGrid]:
    """Every member of set NAME (NumMembers from the info file, else every
    NAME_MMMM.dat present from 0000 on)."""
    d = find_set(name, dirname)
    ipath = os.path.join(d, name + ".info")
    info = read_info(ipath) if os.path.isfile(ipath) else {}
    n = info.get("NumMembers")
    out = []
    m = 0
    while n is None or m < int(n):
        p = os.path.join(d, "%s_%04d.dat" % (name, m))
        if not os.path.isfile(p):
            if n is None:
                break
            raise FormatError("%s: member file missing (NumMembers = %s)" % (p, n))
        out.append(read_member(p, info))
        m += 1
    if not out:
        raise FormatError("set %r has no member files" % name)
    return out


def _fmt(v: np.ndarray) -> str:
    return " ".join(repr(float(t)) for t in v)


def write_set(dirname: str, name: str, members, info: dict | None = None) -> str:
    """Write members (objects with pids, x, q2, q_off, xf and optional
    as_q2 / as_val) as set NAME under dirname; values are written with full
    FP64 precision.  Returns the set's folder."""
    d = os.path.join(dirname, name)
    os.makedirs(d, exist_ok=True)
    m0 = members[0]
    meta = {"Format": "lhagrid1", "NumMembers": len(members),
            "Flavors": [int(p) for p in m0.pids]}
    aq = getattr(m0, "as_q2", None)
    if aq is not None and len(aq):
        meta["AlphaS_Type"] = "ipol"
        meta["AlphaS_Qs"] = [float(v) for v in np.sqrt(np.asarray(aq, dtype=np.float64))]
        meta["AlphaS_Vals"] = [float(v) for v in np.asarray(m0.as_val, dtype=np.float64)]
    meta.update(info or {})
    with open(os.path.join(d, name + ".info"), "w") as fh:
        yaml.safe_dump(meta, fh, default_flow_style=None, sort_keys=False)
    for k, m in enumerate(members):
        xf = np.asarray(m.xf, dtype=np.float64)
        q_off = np.asarray(m.q_off)
        q = np.sqrt(np.asarray(m.q2, dtype=np.float64))
        with open(os.path.join(d, "%s_%04d.dat" % (name, k)), "w") as fh:
            fh.write("PdfType: %s\nFormat: lhagrid1\n---\n" % ("central" if k == 0 else "replica"))
            for s in range(q_off.size - 1):
                a, b = int(q_off[s]), int(q_off[s + 1])
                fh.write(_fmt(m.x) + "\n" + _fmt(q[a:b]) + "\n")
                fh.write(" ".join(str(int(p)) for p in m.pids) + "\n")
                blk = xf[:, :, a:b].transpose(1, 2, 0).reshape(-1, xf.shape[0])
                for row in blk:
                    fh.write(_fmt(row) + "\n")
                fh.write("---\n")
    return d
