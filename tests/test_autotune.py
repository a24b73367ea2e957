"""Host logic of the autotuner: the incumbent configuration stays unless a
challenger is more than 3 % faster, and per-size winners merge into table
entries by size range."""
from paper_1507_02087_amd.autotune import MARGIN, pick, table_entries


def test_incumbent_kept_within_margin():
    assert MARGIN == 1.03
    assert pick({1: 1.00, 2: 0.98}, 1) == 1          # 2 % faster: noise
    assert pick({1: 1.00, 2: 0.971}, 1) == 1         # just inside the margin
    assert pick({1: 1.00, 2: 0.96}, 1) == 2          # 4 % faster: replaces it
    assert pick({1: 1.00, 2: 0.96, 3: 0.90}, 2) == 3
    assert pick({1: 1.00, 2: 1.10}, 7) == 1          # incumbent not timed


def test_table_entries_merge_by_size():
    cfgs = [{"id": 1, "name": "A"}, {"id": 2, "name": "B"}]
    res = [dict(n=n, precision="fp32", best=b)
           for n, b in [(64, 1), (128, 1), (256, 2), (512, 2), (1024, 1)]]
    e = table_entries(res, cfgs)
    assert e == [dict(precision="fp32", n_max=192, name="A"),
                 dict(precision="fp32", n_max=768, name="B"),
                 dict(precision="fp32", n_max=1536, name="A")]
