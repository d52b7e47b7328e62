"""Host-side logic of the Python binding (no GPU): column-major layout
helpers and the carving of a batch's outputs from one allocation."""
import torch

import paper_2603_13532_amd as tsk


def test_fortran_layout_helpers():
    a = torch.arange(24.0).reshape(2, 3, 4)
    f = tsk.fortran(a)
    assert torch.equal(f, a) and tsk.is_fortran(f) and f.stride() == (1, 2, 6)
    assert tsk.fortran(f) is f
    e = tsk.empty_fortran((5, 7), torch.float32, "cpu")
    assert e.shape == (5, 7) and e.stride() == (1, 5)


def test_carve_fortran_views_are_disjoint_aligned_and_column_major():
    shapes = [(100, 13), (13, 13, 13), (1,), (7, 3), (64,)]
    for dt in (torch.float64, torch.float32):
        views = tsk.carve_fortran(shapes, dt, "cpu")
        base = views[0].untyped_storage().data_ptr()
        spans = []
        for v, sh in zip(views, shapes):
            assert tuple(v.shape) == sh and tsk.is_fortran(v)
            assert (v.data_ptr() - base) % 256 == 0
            assert v.untyped_storage().data_ptr() == base
            spans.append((v.data_ptr(), v.data_ptr() + v.numel() * v.element_size()))
        spans.sort()
        assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
        for i, v in enumerate(views):  # writes land in their own view only
            v.fill_(i)
        for i, v in enumerate(views):
            assert torch.all(v == i)


def _struct(m):
    """The fields a marshal hands to the library, read back through its
    pointers (each core and factor as the values at its address, which must
    be its column-major layout)."""
    import ctypes
    S, d = m.sum, m.sum.order
    s = S.num_terms
    ranks = [S.ranks[i] for i in range(s * d)]
    dims = [S.dims[i] for i in range(d)]

    def at(p, n):
        return list((ctypes.c_double * n).from_address(p))
    cores, factors = [], []
    for i in range(s):
        r = ranks[i * d:(i + 1) * d]
        n = 1
        for x in r:
            n *= x
        cores.append(at(S.cores[i], n))
        factors += [at(S.factors[i * d + k], dims[k] * r[k]) for k in range(d)]
    return (d, s, dims, ranks, cores, factors,
            None if not S.coeffs else [S.coeffs[i] for i in range(s)], S.dtype,
            m.spec.kind, m.spec.sizes[0], m.dims, m.d, m.s)


def _colmajor(t):
    return t.permute(*reversed(range(t.dim()))).reshape(-1).tolist()


def test_batched_marshal_matches_one_marshal_per_sum():
    g = torch.Generator().manual_seed(5)
    shared = torch.randn(30, 4, generator=g, dtype=torch.float64)

    def term(dims, ranks, reuse):
        core = torch.randn(*ranks, generator=g, dtype=torch.float64)
        us = [torch.randn(n, r, generator=g, dtype=torch.float64) for n, r in zip(dims, ranks)]
        if reuse:
            us[0] = shared
        return core, us

    sums = []
    for i, (dims, nterms) in enumerate([((30, 9, 7), 3), ((30, 5, 6, 4), 2), ((30, 8), 4),
                                        ((30, 9, 7), 1)]):
        ts = [term(dims, [4] + [2 + (i + j + k) % 3 for k in range(len(dims) - 1)], j % 2 == 0)
              for j in range(nterms)]
        x = {"cores": [c for c, _ in ts], "factors": [us for _, us in ts]}
        if i % 2:
            x["coeffs"] = [0.5 + j for j in range(nterms)]
        sums.append(x)
    # a row-major core and a transposed factor are laid out column-major
    sums[0]["cores"][1] = sums[0]["cores"][1].permute(2, 1, 0).contiguous().permute(2, 1, 0)
    sums[2]["factors"][0][1] = sums[2]["factors"][0][1].t().contiguous().t()
    seen = {}
    one = [tsk._Marshal(x["cores"], x["factors"], x.get("coeffs"), "krp", [1], 0, None,
                        "fp64", "fp64", "auto", seen) for x in sums]
    many = tsk._Marshal.many(sums)
    got = [_struct(m) for m in many]
    assert got == [_struct(m) for m in one]
    for st, x in zip(got, sums):  # and the values are the tensors', column-major
        assert st[4] == [_colmajor(c) for c in x["cores"]]
        assert st[5] == [_colmajor(u) for us in x["factors"] for u in us]
        assert st[6] == x.get("coeffs")
    # a tensor shared between terms and sums is laid out once
    assert many[0].sum.factors[0] == many[3].sum.factors[0] == many[0].sum.factors[6]


def test_batched_marshal_rejects_what_the_constructor_rejects():
    c = torch.zeros(3, 2, dtype=torch.float64)
    u = [torch.zeros(10, 3, dtype=torch.float64), torch.zeros(8, 2, dtype=torch.float64)]
    ok = {"cores": [c], "factors": [u]}
    bad = [
        {"cores": [c], "factors": [[u[0], torch.zeros(8, 5, dtype=torch.float64)]]},
        {"cores": [c, c], "factors": [u, [torch.zeros(11, 3, dtype=torch.float64), u[1]]]},
        {"cores": [c], "factors": [u[:1]]},
        {"cores": [c], "factors": [[u[0].float(), u[1]]]},
        {"cores": [c, c], "factors": [u]},
    ]
    for b in bad:
        for sums in ([b], [ok, b]):
            try:
                tsk._Marshal.many(sums)
            except ValueError:
                continue
            raise AssertionError(f"accepted {b}")
    for b in bad[:4]:
        try:
            tsk._Marshal(b["cores"], b["factors"], None, "krp", [1], 0, None, "fp64", "fp64",
                         "auto")
        except ValueError:
            continue
        raise AssertionError(f"constructor accepted {b}")
