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
