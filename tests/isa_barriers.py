"""Barrier/loop check of gfx950 assembly built from this repository.

Every loop that contains s_barrier (directly or in a nested loop) must close
with a back edge that keeps the wave's lanes together.  A latch that removes
lanes from exec (``s_andn2_b64 exec, exec, ...``) means some lanes of a wave
leave the loop while the others go round again and pass its barrier without
them: a workgroup then proceeds on stale shared state, which shows up as a hang.
The compiler produces that shape when a barrier sits in control flow it cannot
prove uniform, so the kernels broadcast such values with readfirstlane."""
import re, sys

def kernels(lines):
    cur, body = None, []
    for ln in lines:
        m = re.match(r"^(_Z\w+):", ln)
        if m:
            if cur: yield cur, body
            cur, body = m.group(1), []
        elif cur:
            if ln.strip().startswith(".Lfunc_end"):
                yield cur, body; cur, body = None, []
            else:
                body.append(ln)
    if cur: yield cur, body

def check(body):
    blocks, order, inner, parent_of_header = {}, [], {}, {}
    cur = "entry"; blocks[cur] = []; order.append(cur); inner[cur] = None
    pending_ann = None
    for ln in body:
        m = re.match(r"^\.L(BB\d+_\d+):\s*(;.*)?$", ln) or re.match(r"^; %bb\.(\d+):\s*(;.*)?$", ln)
        if m:
            name = m.group(1) if ln.startswith(".L") else "bb" + m.group(1)
            cur = name; blocks[cur] = []; order.append(cur)
            ann = m.group(2) or ""
            inner[cur] = None
            h = re.search(r"Header=(BB\d+_\d+)", ann)
            if h: inner[cur] = h.group(1)
            p = re.search(r"Parent Loop (BB\d+_\d+)", ann)
            if p: inner[cur] = p.group(1); parent_of_header.setdefault(cur, p.group(1))
            continue
        s = ln.strip()
        if "This Loop Header" in s or "This Inner Loop Header" in s:
            # annotation line belongs to the current block: it heads a loop
            parent_of_header.setdefault(cur, inner.get(cur))
            inner[cur] = cur
            continue
        if s.startswith(";") or not s:
            continue
        blocks[cur].append(s)
    headers = set(b for b in order if inner.get(b) == b)
    def loops_of(b):
        out, h = [], inner.get(b)
        seen = set()
        while h and h not in seen:
            seen.add(h); out.append(h)
            h = parent_of_header.get(h)
            if h == out[-1]: break
        return out
    has_bar = {h: False for h in headers}
    for b in order:
        if any(i.startswith("s_barrier") for i in blocks[b]):
            for h in loops_of(b): has_bar[h] = True
    bad = []
    for h in headers:
        if not has_bar.get(h): continue
        members = [b for b in order if h in loops_of(b)]
        idx = order.index(h)
        for b in members:
            ins = blocks[b]
            to_h = any(re.search(r"\.L%s\b" % h, i) for i in ins if i.startswith("s_cbranch") or i.startswith("s_branch"))
            falls = order.index(b) == idx - 1
            if not (to_h or falls): continue
            if any(i.startswith("s_andn2_b64 exec, exec") for i in ins):
                bad.append((h, b))
    return bad

if __name__ == "__main__":
    lines = open(sys.argv[1]).read().splitlines()
    nbad = 0
    for k, body in kernels(lines):
        bad = check(body)
        nbad += bool(bad)
        print(("BAD " if bad else "ok  ") + k[:70], bad[:4])
    sys.exit(1 if nbad else 0)
