"""The autotuner's search logic on a model context (no GPU): each knob is
timed over the kernels it moves work between.

The model is the city frame that answers the G-buffer queries: lane refill
makes the shadow launch itself faster than the batched launch with its half
of the query batch, but moves the whole batch into the trace launch, so the
two traversals together are slower.  Tuning shadow_refill on the shadow
kernels alone would pick refill; the tuner must keep batches."""
import types

from paper_2009_10796_amd import autotune


class ModelCtx:
    """Kernel times (ms) as a function of the tuning, accumulated per frame
    while profiling is on, read back as profile_read does: name -> (launches,
    total ms)."""

    def __init__(self, queries=True):
        self.t = dict(trace_blocks=0, shadow_blocks=0, shade_blocks=0, blend_blocks=0, shadow_refill=0,
                      blend_rsplit=0, query_shadow=500)
        self.queries = queries
        self.on = False
        self.acc = {}
        self.torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))

    def set_tuning(self, **kw):
        self.t.update(kw)

    def profile(self, enable=True):
        self.on = enable

    def profile_read(self, reset=True):
        out = dict(self.acc)
        if reset:
            self.acc = {}
        return out

    def kernels(self):
        t = self.t
        query = 0.050 if self.queries else 0.0
        share = 0.0 if t["shadow_refill"] > 0 else t["query_shadow"] / 1000.0
        ks = {}
        # a small penalty away from an even split makes 500 the best share
        ks["trace_query" if self.queries else "trace"] = 0.040 + query * (1.0 - share) + 0.004 * abs(share - 0.5)
        if t["shadow_refill"] > 0:
            ks["shadow_refill"] = 0.082
        else:
            ks["shadow_query" if self.queries else "shadow"] = 0.060 + query * share
        ks["shade"] = 0.008
        ks["blend_mma"] = 0.014
        return ks

    def step(self, rotation):
        if not self.on:
            return
        for k, ms in self.kernels().items():
            n, tot = self.acc.get(k, (0, 0.0))
            self.acc[k] = (n + 1, tot + ms)


def test_refill_is_timed_with_the_trace_it_moves_queries_into():
    ctx = ModelCtx(queries=True)
    chosen = autotune.autotune(ctx, [None] * 4, frames_per_candidate=2, cu=256, step=ctx.step)
    assert chosen["shadow_refill"] == 0, chosen
    assert chosen["query_shadow"] == 500, chosen
    # the report holds every candidate's time over both traversals
    rep = ctx.tuning_report["shadow_refill"]
    assert set(rep) == {"0", "4", "8", "16", "32"}
    assert rep["0"] < rep["8"]


def test_refill_wins_where_it_is_faster_overall():
    # plain frames whose shadow rays are faster with lane refill (0.050
    # against 0.060 ms batched): the trace does not change, so refill wins
    ctx = ModelCtx(queries=False)
    base = ctx.kernels

    def faster_refill():
        ks = base()
        if "shadow_refill" in ks:
            ks["shadow_refill"] = 0.050
        return ks

    ctx.kernels = faster_refill
    chosen = autotune.autotune(ctx, [None] * 4, frames_per_candidate=2, cu=256, step=ctx.step)
    assert chosen["shadow_refill"] in (4, 8, 16, 32), chosen
    assert "query_shadow" not in chosen      # plain frames do not tune the query split


def test_saved_tuning_applies_to_another_context(tmp_path):
    ctx = ModelCtx(queries=True)
    chosen = autotune.autotune(ctx, [None] * 4, frames_per_candidate=1, cu=256, step=ctx.step)
    path = tmp_path / "sub" / "tuning.json"
    autotune.save(chosen, str(path), "model-city", ctx.tuning_report)
    loaded = autotune.load(str(path))
    assert loaded == chosen and all(isinstance(v, int) for v in loaded.values())
    other = ModelCtx(queries=True)
    autotune.apply(other, loaded)
    assert {k: other.t[k] for k in loaded} == chosen


def test_knob_candidates():
    assert autotune.candidates(256, "shadow_refill") == [0, 4, 8, 16, 32]
    assert autotune.candidates(256, "blend_rsplit") == [4, 2, 1]
    assert autotune.candidates(256, "query_shadow") == [0, 250, 500, 750]
    # grids: 0 (one workgroup per work unit) and multiples of the compute units
    assert autotune.candidates(256, "trace_blocks") == [0, 256, 512, 1024, 2048, 4096]
