"""Host-side measurement helpers of bench.py (no GPU): the dispatch-overlap
summary behind the serving profile, on hand-made kernel traces whose answers
are known."""
import bench


def row(start, end, grid, stream=0, block=1024):
    return {"Start_Timestamp": str(start), "End_Timestamp": str(end), "Grid_Size_X": str(grid * block),
            "Workgroup_Size_X": str(block), "Stream_Id": str(stream)}


def test_back_to_back_dispatches_do_not_overlap():
    o = bench.overlap_stats([row(0, 10, 64), row(10, 25, 192, 1), row(25, 30, 64, 2)])
    assert o["any_ns"] == 30 and o["multi_ns"] == 0
    assert o["most"] == 1 and o["most_workgroups"] == 192
    assert o["cover_ns"] == {1: 30}


def test_overlapping_and_nested_dispatches():
    # [0,100) 64 wg; [20,60) 128 wg; [40,50) 64 wg; [150,160) 64 wg
    o = bench.overlap_stats([row(0, 100, 64, 0), row(20, 60, 128, 1), row(40, 50, 64, 2), row(150, 160, 64, 0)])
    assert o["cover_ns"] == {1: 20 + 40 + 10, 2: 20 + 10, 3: 10}
    assert o["any_ns"] == 110 and o["multi_ns"] == 40
    assert o["most"] == 3 and o["most_workgroups"] == 256
    assert o["grids"] == [64, 128] and o["streams"] == ["0", "1", "2"]


def test_empty_trace():
    o = bench.overlap_stats([])
    assert o["any_ns"] == 0 and o["most"] == 0 and o["most_workgroups"] == 0
