"""Host replay of a prepared device schedule (test infrastructure).

Executes, with numpy, exactly the launch list the library would enqueue
(permutations through their tables, gathered batched GEMMs through their
instance maps, finalize, level sums), on the constant bytes the library would
upload.  This checks the planner and the schedule builder on a machine without
a GPU; it shares no code with the oracle and does not replace the GPU parity
tests, which run the kernels themselves.
"""
import numpy as np


def _deposit_of(x, pos):
    o = np.zeros_like(x)
    for j, p in enumerate(pos):
        o |= ((x >> j) & 1) << p
    return o


def _deposit(count, pos):
    return _deposit_of(np.arange(count, dtype=np.int64), pos)


def _overlap(x, y):
    return x[0] == y[0] and x[1] < y[2] and y[1] < x[2]


class Sim:
    def __init__(self, desc, const_bytes):
        self.desc = desc
        self.const = np.array(const_bytes, dtype=np.uint8, copy=True)
        extra = max(0, desc["const_bytes"] - self.const.size)
        if extra:
            self.const = np.concatenate([self.const, np.zeros(extra, np.uint8)])
        self.work = np.zeros(max(256, desc["work_bytes"]), dtype=np.uint8)
        self.partials = {}      # split partial tiles written and not yet reduced

    def region(self, ref):
        return self.const if ref[0] == 0 else self.work

    def _ref(self, ref):
        # the FP64 pass lives after the FP32 work region
        if ref[0] == 2:
            return [1, ref[1] + self.desc["work1_bytes"]]
        return ref

    def view(self, ref, dtype, count, extra_off=0):
        ref = self._ref(ref)
        buf = self.region(ref)
        off = ref[1] + extra_off
        nbytes = np.dtype(dtype).itemsize * count
        assert off >= 0 and off + nbytes <= buf.size, ("out of bounds", ref, count, buf.size)
        return buf[off:off + nbytes].view(dtype)

    def cview(self, off, dtype, count):
        return self.view([0, off], dtype, count)

    def perm(self, L):
        dt = np.complex128 if L["fp64"] else np.complex64
        r, tb, n = L["r"], L["tb"], L["n_inst"]
        tsize = 1 << tb
        table = self.view(L["table"], np.int32, 3 * tsize)
        ld_in, ld_pos, st_out = table[:tsize], table[tsize:2 * tsize], table[2 * tsize:]
        size = 1 << r
        src = self.view(L["a"], dt, n * size).reshape(n, size)
        dst = self.view(L["c"], dt, n * size).reshape(n, size)
        nh = r - tb
        hs = np.arange(1 << nh, dtype=np.int64)
        in_base = np.zeros_like(hs)
        out_base = np.zeros_like(hs)
        for i in range(nh):
            bit = (hs >> i) & 1
            in_base |= bit << L["high_in"][i]
            out_base |= bit << L["high_out"][i]
        # tile element e sits at LDS position e; loads put src[in_base+ld_in[l]] at ld_pos[l]
        lds_src = np.empty(tsize, dtype=np.int64)
        lds_src[ld_pos] = ld_in
        in_idx = (in_base[:, None] + lds_src[None, :]).reshape(-1)
        out_idx = (out_base[:, None] + st_out[None, :].astype(np.int64)).reshape(-1)
        assert in_idx.min() >= 0 and in_idx.max() < size and out_idx.max() < size
        assert np.unique(out_idx).size == size
        tmp = np.empty_like(src)
        tmp[:, out_idx] = src[:, in_idx]
        dst[...] = tmp

    def gemm(self, L, c_extra=0):
        if L.get("gather"):
            return self.gemm_gather(L, c_extra)
        dt = np.complex128 if L["fp64"] else np.complex64
        m, n, k = 1 << L["m_log"], 1 << L["n_log"], 1 << L["k_log"]
        ni = L["n_inst"]

        def idx(mode, ref):
            if mode == 0:
                return np.arange(ni)
            if mode == 1:
                return np.zeros(ni, dtype=np.int64)
            return self.view(ref, np.int32, ni).astype(np.int64)
        ia, ib = idx(L["ia_mode"], L["ia"]), idx(L["ib_mode"], L["ib"])
        na, nb = int(ia.max()) + 1, int(ib.max()) + 1
        A = self.view(L["a"], dt, na * L["strideA"]).reshape(na, L["strideA"])[:, :m * k]
        B = self.view(L["b"], dt, nb * L["strideB"]).reshape(nb, L["strideB"])[:, :k * n]
        A = A.reshape(na, k, m).transpose(0, 2, 1) if L["transA"] else A.reshape(na, m, k)
        B = B.reshape(nb, n, k).transpose(0, 2, 1) if L["transB"] else B.reshape(nb, k, n)
        Cv = self.view(L["c"], dt, ni * m * n, c_extra).reshape(ni, m, n)
        Cv[...] = np.matmul(A[ia].astype(np.complex128), B[ib].astype(np.complex128)).astype(dt)

    def gemm_gather(self, L, c_extra=0, dt=np.complex64):
        """Operands read in stored order: logical bit j of the row / inner /
        column index sits at the stored position a_row[j] / a_k[j] (b_k[j]) /
        b_col[j]; instance i starts at offset oa[i] (ob[i])."""
        m, n, k = 1 << L["m_log"], 1 << L["n_log"], 1 << L["k_log"]
        ni = L["n_inst"]

        def deposit(count, pos):
            x = np.arange(count, dtype=np.int64)
            o = np.zeros(count, dtype=np.int64)
            for j, p in enumerate(pos):
                o |= ((x >> j) & 1) << p
            return o
        assert len(L["a_row"]) == L["m_log"] and len(L["b_col"]) == L["n_log"]
        assert len(L["a_k"]) == L["k_log"] == len(L["b_k"])
        for pos in (L["a_row"] + L["a_k"], L["b_k"] + L["b_col"]):
            assert len(set(pos)) == len(pos), "stored positions must be distinct"
        oa = self.view(L["oa"], np.int64, ni)
        ob = self.view(L["ob"], np.int64, ni)
        ra, ka = deposit(m, L["a_row"]), deposit(k, L["a_k"])
        kb, cb = deposit(k, L["b_k"]), deposit(n, L["b_col"])
        a_idx = oa[:, None, None] + ra[None, :, None] + ka[None, None, :]
        b_idx = ob[:, None, None] + kb[None, :, None] + cb[None, None, :]
        assert a_idx.min() >= 0 and b_idx.min() >= 0
        A = self.view(L["a"], dt, int(a_idx.max()) + 1)
        B = self.view(L["b"], dt, int(b_idx.max()) + 1)
        Cv = self.view(L["c"], dt, ni * m * n, c_extra).reshape(ni, m, n)
        Cv[...] = np.matmul(A[a_idx].astype(np.complex128), B[b_idx].astype(np.complex128)).astype(dt)

    def finalize(self, L, root_refs, root64_refs):
        nt, ncl = L["n_terms"], L["n_clusters"]
        live = self.cview(L["live_index"], np.int32, max(1, nt))[:nt]
        nlive = int((live >= 0).sum())
        ridx = self.cview(L["root_idx"], np.int32, max(1, nlive * ncl))[:nlive * ncl].reshape(nlive, ncl) \
            if nlive else np.zeros((0, ncl), np.int32)
        w = self.cview(L["w"], np.float64, max(1, nt))[:nt]
        x = self.cview(L["x_out"], np.float64, max(1, nt))
        amp = self.cview(L["amp_out"], np.complex64, max(1, nt))
        sc = complex(*L["scalar"])
        for t in range(nt):
            li = live[t]
            if li < 0:
                x[t] = 0
                amp[t] = 0
                continue
            a = sc
            for c in range(ncl):
                j = int(ridx[li, c])
                if t == L["zero_term"]:
                    a *= complex(self.view(root64_refs[c], np.complex128, j + 1)[j])
                else:
                    a *= complex(self.view(root_refs[c], np.complex64, j + 1)[j])
            x[t] = w[t] * (a.real if L.get("re_value") else abs(a) ** 2)
            amp[t] = a

    def level_sum(self, L):
        n_levels = L["n_levels"]
        starts = self.cview(L["starts"], np.int64, n_levels + 1)
        x = self.cview(L["x_out"], np.float64, int(starts[-1]) if starts[-1] else 1)
        out = self.cview(L["sums"], np.float64, 2 * n_levels)
        for u in range(n_levels):
            seg = x[starts[u]:starts[u + 1]]
            out[2 * u] = float(np.sum(seg.astype(np.float64)))
            out[2 * u + 1] = 0.0

    def slot_fill(self, L, term):
        n = L["n"]
        noise = self.cview(L["noise"], np.int32, max(1, n))[:n]
        dst = self.cview(L["dst"], np.int64, max(1, n))[:n]
        N = L["n_noise"]
        bank = self.cview(L["bank"], np.float32, N * 32 + 8)
        pat = self.cview(L["pattern"], np.int8, (term + 1) * N)
        for i in range(n):
            s = int(noise[i])
            ch = int(pat[term * N + s])
            self.view([0, int(dst[i])], np.float32, 8)[:] = bank[(s * 4 + ch) * 8:(s * 4 + ch) * 8 + 8]

    def run(self, live_terms_per_plan=None):
        d = self.desc
        # slot-free steps first: the library runs them once when the schedule is bound
        for L in d["launches"]:
            if L["phase"] == "const":
                self.exec(L)
        batch = [L for L in d["launches"] if L["phase"] in ("batch", "batch64")]
        plain = [L for L in d["launches"] if L["phase"] == "plain"]
        tail = [L for L in d["launches"] if L["phase"] == "tail"]
        for L in batch:
            self.exec(L)
        assert not self.partials, ("partial tiles never reduced", sorted(self.partials)[:4])
        if d["mode"] == 1:
            for t in range(d["plain_terms"]):
                term = live_terms_per_plan[0][t]
                for L in plain:
                    if L["kind"] == 4:
                        self.slot_fill(L, term)
                    elif L["kind"] == 1 and L.get("plain_root"):
                        self.gemm(L, c_extra=8 * t)
                    else:
                        self.exec(L)
        for L in tail:
            pe = d["plans"][L["plan"]]
            if L["kind"] == 2:
                self.finalize(L, pe["root32"], pe["root64"])
            elif L["kind"] == 3:
                self.level_sum(L)

    def group(self, L):
        """One grouped launch: every job is an independent gathered contraction
        (same addressing as the gathered GEMM); jobs of one launch never write
        what another job of it reads."""
        def dtype_of(jb):
            # a level's launch may hold the FP64 dominant-term pass's jobs too
            return np.complex128 if jb.get("fp64", L["fp64"]) else np.complex64
        spans = []
        for jb in L["jobs"]:
            spans.append(self._job_spans(jb, np.dtype(dtype_of(jb)).itemsize))
        for i, (wi, _) in enumerate(spans):
            for j, (wj, rj) in enumerate(spans):
                for other in ([wj] if i != j else []) + rj:
                    assert not _overlap(wi, other), ("grouped jobs race", i, j, wi, other)
        for jb in L["jobs"]:
            self.gemm_gather(jb, dt=dtype_of(jb))

    def _job_spans(self, jb, esz):
        """(write span, [read spans]) of one grouped job, as (region, start, end) bytes."""
        m, n, k = 1 << jb["m_log"], 1 << jb["n_log"], 1 << jb["k_log"]
        ni = jb["n_inst"] if "n_inst" in jb else jb["ns"]
        oa = self.view(jb["oa"], np.int64, ni)
        ob = self.view(jb["ob"], np.int64, ni)
        amax = int(oa.max()) + sum(1 << p for p in jb["a_row"] + jb["a_k"])
        bmax = int(ob.max()) + sum(1 << p for p in jb["b_k"] + jb["b_col"])

        def span(ref, lo, hi):
            r = self._ref(ref)
            return (min(r[0], 1), r[1] + lo * esz, r[1] + hi * esz)
        return (span(jb["c"], 0, ni * m * n),
                [span(jb["a"], int(oa.min()), amax + 1), span(jb["b"], int(ob.min()), bmax + 1)])

    TILE = np.dtype([("job", "<i4"), ("cnt", "<i4"), ("s0", "<i8"), ("tm0", "<i8"), ("tn0", "<i8"),
                     ("kpart", "<i4"), ("pair", "<i4")])

    def mgroup(self, L):
        """Grouped matrix-core launch, tile by tile as the kernel builds its
        row / column offset tables; every output element of every job must be
        written exactly once, and no job may write what another job reads."""
        bm, bn = L["bm"], L["bn"]
        dt = np.complex128 if L["fp64"] else np.complex64
        esz = np.dtype(dt).itemsize
        tiles = self.view(L["tiles"], np.uint8, L["n_tiles"] * self.TILE.itemsize).view(self.TILE)
        jobs = L["jobs"]
        spans = [self._job_spans(jb, esz) for jb in jobs]
        for i, (wi, _) in enumerate(spans):
            for j, (wj, rj) in enumerate(spans):
                for other in ([wj] if i != j else []) + rj:
                    assert not _overlap(wi, other), ("grouped jobs race", i, j, wi, other)
        ctx = [self._mjob_ctx(jb, dt) for jb in jobs]
        for t in tiles:
            jb = jobs[t["job"]]
            m, n, k, oa, ob, oc, A, B, C, hits, ka, kb = ctx[t["job"]]
            S = int(jb.get("ksplit", 1))
            if S > 1:
                # the inner sum of a tile group is split in S equal parts of whole
                # 8-term chunks; each block leaves its partial tile
                assert S & (S - 1) == 0 and k >= 8 and (k // 8) % S == 0 and S <= bm * bn, ("split", S, k)
                assert 0 <= int(t["kpart"]) < S, ("part index", int(t["kpart"]), S)
                h = k // S
                sel = slice(int(t["kpart"]) * h, (int(t["kpart"]) + 1) * h)
                ka, kb = ka[sel], kb[sel]
            ok_r, rc, ok_c, cc = self._tile_out(jb, t, bm, bn, m, n, oc)
            ra, cb = self._tile_in(jb, t, bm, bn, m, n, oa, ob)
            ra, cb = ra[ok_r], cb[ok_c]
            At = A[ra[:, None] + ka[None, :]].astype(np.complex128)
            Bt = B[kb[:, None] + cb[None, :]].astype(np.complex128)
            part = (At @ Bt).astype(dt).reshape(-1)
            if S > 1:
                # row-major [bm][bn] partial tile of group `pair`, part `kpart`
                slot = int(t["pair"]) * S + int(t["kpart"])
                P = self.view(jb["partial"], dt, (slot + 1) * bm * bn)[slot * bm * bn:]
                rows, cols = np.nonzero(ok_r)[0], np.nonzero(ok_c)[0]
                P[(rows[:, None] * bn + cols[None, :]).reshape(-1)] = part
                self.partials[(tuple(jb["partial"]), slot)] = (rows, cols)
                continue
            idx = (rc[ok_r][:, None] + cc[ok_c][None, :]).reshape(-1)
            C[idx] = part
            np.add.at(hits, idx, 1)
        for q, cx in enumerate(ctx):
            if int(jobs[q].get("ksplit", 1)) == 1:
                assert cx[9].min() == 1 and cx[9].max() == 1, ("output coverage", q, cx[9].min(), cx[9].max())

    def mreduce(self, L):
        """Split-sum reduction after a grouped launch: block (group, part) adds
        the rows [part bm / S, (part + 1) bm / S) of the group's S partial tiles
        in part order and writes C; every output of every split job exactly once."""
        bm, bn = L["bm"], L["bn"]
        dt = np.complex128 if L["fp64"] else np.complex64
        tiles = self.view(L["tiles"], np.uint8, L["n_tiles"] * self.TILE.itemsize).view(self.TILE)
        jobs = L["jobs"]
        ctx = [self._mjob_ctx(jb, dt) for jb in jobs]
        for t in tiles:
            jb = jobs[t["job"]]
            S = int(jb.get("ksplit", 1))
            if S == 1:
                continue
            m, n, k, oa, ob, oc, A, B, C, hits, ka, kb = ctx[t["job"]]
            g, h = int(t["pair"]), int(t["kpart"])
            P = self.view(jb["partial"], dt, (g + 1) * S * bm * bn)[g * S * bm * bn:].reshape(S, bm, bn)
            ok_r, rc, ok_c, cc = self._tile_out(jb, t, bm, bn, m, n, oc)
            cols = np.nonzero(ok_c)[0]
            for q in range(S if h == 0 else 0):      # every part wrote exactly these elements
                got = self.partials.pop((tuple(jb["partial"]), g * S + q), None)
                assert got is not None, ("missing partial tile", g, q)
                assert np.array_equal(got[0], np.nonzero(ok_r)[0]) and np.array_equal(got[1], cols)
            if S > bm:
                # more parts than rows: block h takes elements [h E, (h + 1) E) of the
                # row-major tile (E = bm bn / S), summed over the parts in FP64
                E = bm * bn // S
                flat = np.arange(h * E, (h + 1) * E)
                ri, ci = flat // bn, flat % bn
                keep = ok_r[ri] & ok_c[ci]
                ri, ci = ri[keep], ci[keep]
                acc = P[:, ri, ci].astype(np.complex128).sum(0).astype(dt)
                idx = rc[ri] + cc[ci]
                C[idx] = acc
                np.add.at(hits, idx, 1)
                continue
            rows = np.arange(h * (bm // S), (h + 1) * (bm // S))
            rows = rows[ok_r[rows]]
            acc = P[0][rows[:, None], cols[None, :]]
            for q in range(1, S):
                acc = (acc + P[q][rows[:, None], cols[None, :]]).astype(dt)
            idx = (rc[rows][:, None] + cc[cols][None, :]).reshape(-1)
            C[idx] = acc.reshape(-1)
            np.add.at(hits, idx, 1)
        for q, cx in enumerate(ctx):
            if int(jobs[q].get("ksplit", 1)) > 1:
                assert cx[9].min() == 1 and cx[9].max() == 1, ("split output coverage", q, cx[9].min(), cx[9].max())

    def _mjob_ctx(self, jb, dt):
        m, n, k = 1 << jb["m_log"], 1 << jb["n_log"], 1 << jb["k_log"]
        ns = jb["ns"]
        oa = self.view(jb["oa"], np.int64, ns)
        ob = self.view(jb["ob"], np.int64, ns)
        oc = self.view(jb["oc"], np.int64, ns)
        amax = int(oa.max()) + sum(1 << p for p in jb["a_row"] + jb["a_k"])
        bmax = int(ob.max()) + sum(1 << p for p in jb["b_k"] + jb["b_col"])
        A = self.view(jb["a"], dt, amax + 1)
        B = self.view(jb["b"], dt, bmax + 1)
        C = self.view(jb["c"], dt, ns * m * n)
        return (m, n, k, oa, ob, oc, A, B, C, np.zeros(ns * m * n, np.int32),
                _deposit(k, jb["a_k"]), _deposit(k, jb["b_k"]))

    @staticmethod
    def _tile_out(jb, t, bm, bn, m, n, oc):
        """Validity and C offsets of a tile's rows and columns (as the kernels'
        offset tables: merge 2 stacks slices along rows, merge 1 along columns)."""
        cnt, s0, tm0, tn0 = int(t["cnt"]), int(t["s0"]), int(t["tm0"]), int(t["tn0"])
        i = np.arange(bm, dtype=np.int64)
        j = np.arange(bn, dtype=np.int64)
        if jb["merge"] == 2:
            seg, r = i >> jb["m_log"], i & (m - 1)
            ok_r = seg < cnt
            rc = oc[s0 + np.minimum(seg, cnt - 1)] + r * n
        else:
            r = tm0 + i
            ok_r = r < m
            rc = (0 if jb["merge"] == 1 else oc[s0]) + r * n
        if jb["merge"] == 1:
            seg, c = j >> jb["n_log"], j & (n - 1)
            ok_c = seg < cnt
            cc = oc[s0 + np.minimum(seg, cnt - 1)] + c
        else:
            c = tn0 + j
            ok_c = c < n
            cc = c
        return ok_r, rc, ok_c, cc

    @staticmethod
    def _tile_in(jb, t, bm, bn, m, n, oa, ob):
        cnt, s0, tm0, tn0 = int(t["cnt"]), int(t["s0"]), int(t["tm0"]), int(t["tn0"])
        i = np.arange(bm, dtype=np.int64)
        j = np.arange(bn, dtype=np.int64)
        if jb["merge"] == 2:
            seg, r = i >> jb["m_log"], i & (m - 1)
            ra = oa[s0 + np.minimum(seg, cnt - 1)] + _deposit_of(r, jb["a_row"])
        else:
            ra = oa[s0] + _deposit_of((tm0 + i) % m, jb["a_row"])
        if jb["merge"] == 1:
            seg, c = j >> jb["n_log"], j & (n - 1)
            cb = ob[s0 + np.minimum(seg, cnt - 1)] + _deposit_of(c, jb["b_col"])
        else:
            cb = ob[s0] + _deposit_of((tn0 + j) % n, jb["b_col"])
        return ra, cb

    def exec(self, L):
        if L["kind"] == 5:
            self.group(L)
            return
        if L["kind"] == 6:
            self.mgroup(L)
            return
        if L["kind"] == 7:
            self.mreduce(L)
            return
        if L["kind"] == 0:
            self.perm(L)
        elif L["kind"] == 1:
            self.gemm(L)
        else:
            raise AssertionError(L["kind"])

    def outputs(self, plan=0):
        pe = self.desc["plans"][plan]
        n = pe["n_terms"]
        x = self.cview(pe["x_out"], np.float64, max(1, n))[:n].copy()
        amp = self.cview(pe["amp_out"], np.complex64, max(1, n))[:n].copy()
        return x, amp
