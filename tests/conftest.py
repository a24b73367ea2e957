import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (minutes); excluded from the quick suite with -m 'not slow'")


def pytest_collection_modifyitems(config, items):
    # GPU tests are skipped (not failed) when no GPU is present; the product
    # path itself never falls back to the CPU.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(autouse=True)
def _replay_scalar_decisions(request, monkeypatch):
    """Every run a GPU test makes through the binding's contexts (and so
    through run_dense / run_batch) is followed by a replay of the run's
    observed orders, polynomial choices and stop on its own returned history
    (tests/stop_replay.py), with the rule set that the context's init,
    set_homo_lumo and set_mcweeny calls selected."""
    if "gpu" not in request.keywords:
        yield
        return
    import inspect
    from types import SimpleNamespace

    import paper_1507_02087_amd as sp2
    from tests import stop_replay

    def wrap_init(cls, name):
        orig = getattr(cls, name)
        sig = inspect.signature(orig)

        def init(self, *a, **k):
            out = orig(self, *a, **k)
            b = sig.bind(self, *a, **k)
            b.apply_defaults()
            g = b.arguments
            self._replay = dict(lmin=g["lambda_min"], lmax=g["lambda_max"],
                                n_occ=g["n_occ"], branch=g["branch"], norm=g["norm"])
            return out
        monkeypatch.setattr(cls, name, init)

    for cls, name in ((sp2.Context, "init_dense"), (sp2.BsrContext, "init_bsr"),
                      (sp2.BatchContext, "batch_init")):
        wrap_init(cls, name)

    orig_hl, orig_mw = sp2.Context.set_homo_lumo, sp2.Context.set_mcweeny

    def set_homo_lumo(self, homo_out, homo_in, lumo_in, lumo_out, accelerate=True):
        orig_hl(self, homo_out, homo_in, lumo_in, lumo_out, accelerate)
        self._replay.update(homo_lumo=(homo_out, homo_in, lumo_in, lumo_out),
                            accelerate=accelerate)

    def set_mcweeny(self, mu, xi=None):
        orig_mw(self, mu, xi)
        self._replay.update(mcweeny=(mu, xi))

    monkeypatch.setattr(sp2.Context, "set_homo_lumo", set_homo_lumo)
    monkeypatch.setattr(sp2.Context, "set_mcweeny", set_mcweeny)

    orig_run, orig_brun = sp2.Context.run, sp2.BatchContext.batch_run

    def run(self):
        st = orig_run(self)
        rp = self._replay
        n, _, _ = self.get_info()
        m = self.get_norm_history() if rp["norm"] != "fro" else []
        res = SimpleNamespace(n=n, status=st, m=m, **self.get_history())
        stop_replay.replay_run(res, rp["lmin"], rp["lmax"], rp["n_occ"], rp)
        return st

    def batch_run(self):
        st = orig_brun(self)
        rp = self._replay
        res = []
        for b in range(len(self._ns)):
            _, stt, it, _ = self.batch_get(b, with_density=False)
            m = self.get_norm_history(b) if rp["norm"] != "fro" else []
            res.append(SimpleNamespace(n=it, status=stt, m=m, **self.batch_history(b)))
        opts = dict(rp)
        if opts.get("mcweeny") is not None:
            mu, xi = opts["mcweeny"]
            if isinstance(mu, (int, float)):
                opts["mcweeny"] = ([mu], None if xi is None else [xi])
        if opts.get("homo_lumo") is not None and isinstance(opts["homo_lumo"][0], (int, float)):
            opts["homo_lumo"] = tuple([x] for x in opts["homo_lumo"])
        stop_replay.replay_batch(res, list(rp["lmin"]), list(rp["lmax"]),
                                 list(rp["n_occ"]), opts)
        return st

    monkeypatch.setattr(sp2.Context, "run", run)
    monkeypatch.setattr(sp2.BatchContext, "batch_run", batch_run)
    yield
