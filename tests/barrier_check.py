"""Report workgroup barriers inside lane-divergent loops in AMDGPU asm.

Loops come from the assembler's own annotations ("in Loop: Header=..."); a
loop is lane-divergent when a block directly in it updates exec with the
loop-exit mask pattern (s_andn2_b64 exec, exec, ...).  A barrier in such a
loop (or in a loop nested in it) can be executed a different number of times
by different wavefronts of a workgroup.
"""
import re, subprocess, sys


def kernels(path):
    s = open(path).read()
    for m in re.finditer(r'^(_Z[^:\s]+):', s, re.M):
        end = s.find('.Lfunc_end', m.end())
        if end > 0:
            yield m.group(1), s[m.end():end].split('\n')


def analyse(lines):
    blocks = []              # [label, innermost header or None, [instrs]]
    parent = {}
    cur = ['entry', None, []]
    blocks.append(cur)
    last_header = None
    for l in lines:
        raw = l.strip()
        m = re.match(r'(\.LBB\d+_\d+):\s*(;.*)?$', raw) or re.match(r'; %bb\.\d+:\s*(;.*)?$', raw)
        if m:
            label = raw.split(':')[0]
            comment = raw.split(';', 1)[1] if ';' in raw else ''
            hdr = None
            mm = re.search(r'in Loop: Header=(BB\d+_\d+)', comment)
            if mm:
                hdr = mm.group(1)
            if 'Loop Header' in comment:
                hdr = label.lstrip('.L')
                last_header = hdr
            cur = [label, hdr, []]
            blocks.append(cur)
            continue
        mm = re.search(r'Parent Loop (BB\d+_\d+)', raw)
        if mm and last_header:
            parent.setdefault(last_header, mm.group(1))
        t = raw.split(';')[0].strip()
        if t:
            cur[2].append(t)
    divergent = set()
    for label, hdr, ins in blocks:
        if hdr and any(re.match(r's_andn2_b(64|32) exec(_lo)?, exec(_lo)?,', t) for t in ins):
            divergent.add(hdr)
    nb, bad = 0, 0
    for label, hdr, ins in blocks:
        for t in ins:
            if t.startswith('s_barrier'):
                nb += 1
                h = hdr
                while h:
                    if h in divergent:
                        bad += 1
                        break
                    h = parent.get(h)
    return nb, bad, len(divergent)


def report(path):
    """[(kernel, barriers, barriers in lane-divergent loops)] for every kernel with a barrier."""
    out = []
    for name, lines in kernels(path):
        nb, bad, _ = analyse(lines)
        if nb:
            out.append((name, nb, bad))
    return out


if __name__ == "__main__":
    ok = True
    for path in sys.argv[1:]:
        for name, nb, bad in report(path):
            dm = subprocess.run(['c++filt', name], capture_output=True, text=True).stdout.strip()
            print(f"{'BAD' if bad else 'ok'}: {bad}/{nb} barriers in lane-divergent loops: {dm[:100]}")
            ok = ok and not bad
    sys.exit(0 if ok else 1)
