"""The z-front scan's evaluation form against the front's definition (host-side model).

The GPU pass (`thickness.hip: front_scan`) does not close groups of equal D one by
one. It takes an entry as soon as its residual exceeds the lane's running maximum,
through t = A + 2 z zc against mz = maxb + z^2 with A = D - zc^2. A later entry of the
same D replaces the lane's last member, and entries are tested four at a time. Both
functions below return the front of one slice, newest member first. The parity tests
check the kernel's output against the oracle. This test checks the algebra and
control flow of the scan form against the definition: by decreasing D, a group of
equal D contributes its largest residual D - dz^2 when that exceeds every residual of
larger D. It runs on random lists (many equal-D groups, D up to the 3D limit 2^18).
"""
import random


def front_by_definition(entries, z):
    """entries: (D, zc) sorted by decreasing (D << 11) | zc."""
    front, maxb = [], 0
    i = 0
    while i < len(entries):
        v = entries[i][0]
        best, best_dz = 0, 0
        while i < len(entries) and entries[i][0] == v:       # one group of equal D
            dz = z - entries[i][1]
            b = v - dz * dz
            if b > best:                                     # strict: the first (larger zc) of equals
                best, best_dz = b, dz
            i += 1
        if best > maxb:
            front.insert(0, (v, best_dz))
            maxb = best
    return front


def front_by_scan_form(entries, z):
    """The kernel's form: (zc, A) pairs padded to a multiple of four with entries no
    slice takes, the D of every fourth entry for the stop test."""
    cnt = len(entries)
    cnt4 = (cnt + 3) & ~3
    pad = -(1 << 30)
    ent = [(zc, v - zc * zc) for (v, zc) in entries] + [(0, pad)] * (cnt4 - cnt)
    dq = [entries[4 * i + 3][0] if 4 * i + 3 < cnt else pad for i in range(cnt4 // 4)]
    z2, zsq = 2 * z, z * z
    mz = zsq
    front, lastv, more, j = [], 0, True, 0
    while more and j < cnt4:
        t = [z2 * ent[j + u][0] + ent[j + u][1] for u in range(4)]
        if max(t) > mz:                                      # some entry of the four is taken
            for u in range(4):
                if t[u] > mz:
                    zc, a = ent[j + u]
                    v = zc * zc + a
                    if v != lastv:
                        front.insert(0, (v, z - zc))
                    else:
                        front[0] = (v, z - zc)               # same D: the larger residual replaces
                    lastv, mz = v, t[u]
        more = mz < dq[j >> 2] + zsq                         # maxb below the D of the fourth
        j += 4
    return front


def _random_list(rng):
    cnt = rng.randint(1, 128)
    vmax = rng.choice([4, 20, 200, 3000, 1 << 18])
    zs = rng.sample(range(1024), cnt)
    ent = {(rng.randint(1, vmax), zc) for zc in zs}
    return sorted(ent, key=lambda e: (e[0] << 11) | e[1], reverse=True)


def test_scan_form_equals_definition():
    rng = random.Random(20250408)
    for _ in range(3000):
        ent = _random_list(rng)
        for z in rng.sample(range(1024), 4):
            assert front_by_scan_form(ent, z) == front_by_definition(ent, z), (ent, z)


def test_scan_form_special_cases():
    # one centre: a front of one member exactly inside its open ball
    assert front_by_scan_form([(10, 5)], 5) == [(10, 0)]
    assert front_by_scan_form([(10, 5)], 8) == [(10, 3)]      # 10 - 9 = 1 > 0
    assert front_by_scan_form([(9, 5)], 8) == []              # 9 - 9 = 0: outside the open ball
    # equal D on both sides of the slice: equal residuals keep the larger zc
    assert front_by_scan_form([(16, 7), (16, 3)], 5) == [(16, -2)]
    # a smaller D nearer the slice joins the front when its residual is larger
    assert front_by_scan_form([(100, 20), (50, 11)], 11) == [(50, 0), (100, -9)]
    assert front_by_definition([(100, 20), (50, 11)], 11) == [(50, 0), (100, -9)]
    # ... and stays out when it is not (residual 9 against 19)
    assert front_by_scan_form([(100, 20), (9, 11)], 11) == [(100, -9)]
