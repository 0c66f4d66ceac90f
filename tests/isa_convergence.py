"""Find loops in gfx950 assembly whose latch narrows EXEC (a divergent exit)
while the loop body holds a cross-lane operation (readfirstlane, bpermute,
s_barrier)."""
import re
CONV = re.compile(r'v_readfirstlane|ds_bpermute|s_barrier')
def check(lines):
    labels = {}
    for i, l in enumerate(lines):
        m = re.match(r'^(\.LBB\d+_\d+):', l)
        if m: labels[m.group(1)] = i
    bad = []
    for i, l in enumerate(lines):
        if 's_andn2_b64 exec, exec' not in l: continue
        nxt = lines[i + 1] if i + 1 < len(lines) else ''
        m = re.search(r'(\.LBB\d+_\d+)', nxt)
        if m and 'execnz' in nxt and labels.get(m.group(1), 10**9) < i:
            lo, hi = labels[m.group(1)], i
        elif m and 'execz' in nxt:
            # falls through into the loop header when lanes remain
            j = i + 2
            while j < len(lines) and not lines[j].startswith('.LBB'): j += 1
            if j >= len(lines): continue
            hdr = re.match(r'^(\.LBB\d+_\d+):', lines[j]).group(1)
            # latch block label: nearest label above i
            k = i
            while k >= 0 and not lines[k].startswith('.LBB'): k -= 1
            latch = re.match(r'^(\.LBB\d+_\d+):', lines[k]).group(1) if k >= 0 else None
            refs = [t for t, x in enumerate(lines) if latch and re.search(re.escape(latch) + r'\b', x) and not x.startswith(latch)]
            lo, hi = j, max(refs + [j])
        else:
            continue
        conv = [x.strip() for x in lines[lo:hi + 1] if CONV.search(x)]
        if conv: bad.append((lo, hi, conv[:2]))
    return bad
