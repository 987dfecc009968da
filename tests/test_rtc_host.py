"""User kernels compiled at run time (Sec. 3.5), host side: definition
errors are reported at definition time (parameter lists, annotations,
compiler messages), and a user kernel is planned like a built-in one
(dry-run contexts: same regions and DAG as the built-in body under the same
annotation).  hipRTC compiles for gfx950 without a GPU."""
import numpy as np
import pytest

import paper_2202_05549_amd as L

STENCIL = r"""
__device__ void stencil(dim3 virtBlockIdx, int n, lt::Vector<float> output, const lt::Vector<float> input) {
    int i = blockDim.x * virtBlockIdx.x + threadIdx.x;
    if (i >= n) return;
    float left = i - 1 >= 0 ? input[i - 1] : 0.0f;
    float right = i + 1 < n ? input[i + 1] : 0.0f;
    output[i] = 0.25f * (left + right) + 0.5f * input[i];
}
"""
PARAMS = [("n", "int"), ("output", np.float32, 1), ("input", np.float32, 1)]
ANN = "global i => read input[i-1:i+1], write output[i]"


def dry(**kw):
    kw.setdefault("device_budget_bytes", 1 << 30)
    return L.Context(dry_run=1, **kw)


def test_defines_and_plans_like_the_builtin():
    n, chunk = 10_000, 1000
    plans = []
    for name in ("user_stencil", "stencil1d_f32"):
        ctx = dry()
        if name == "user_stencil":
            ctx.define_source(name, STENCIL, "stencil", PARAMS, ANN)
        x = ctx.array([n], chunk=[chunk])
        y = ctx.array([n], chunk=[chunk])
        l1 = ctx.launch(name, [n], [16], [2000], args=[n, y, x])
        l2 = ctx.launch(name, [n], [16], [2000], args=[n, x, y])
        tasks = ctx.tasks(l1) + ctx.tasks(l2)
        regions = [[(r.arg, r.mode, tuple(r.lo), tuple(r.hi)) for r in ctx.regions(t.id)] for t in tasks]
        deps = [ctx.deps(t.id) for t in tasks]
        plans.append((regions, deps))
        ctx.close()
    assert plans[0] == plans[1]


def test_compile_error_is_reported_with_the_log():
    ctx = dry()
    bad = STENCIL.replace("output[i] =", "output[i] = undefined_name +")
    with pytest.raises(L.LtError) as e:
        ctx.define_source("bad", bad, "stencil", PARAMS, ANN)
    assert e.value.status == L.LT_ERR_COMPILE
    assert "undefined_name" in str(e.value)
    ctx.close()


def test_signature_mismatch_is_a_compile_error():
    # the wrapper calls the function with the declared parameter list
    ctx = dry()
    with pytest.raises(L.LtError) as e:
        ctx.define_source("two", STENCIL, "stencil", PARAMS[:2], "global i => write output[i]")
    assert e.value.status == L.LT_ERR_COMPILE
    ctx.close()


@pytest.mark.parametrize("params,fn,ann,status", [
    ([("n", "int"), ("n", np.float32, 1)], "stencil", "global i => write n[i]", "INVALID"),   # duplicate name
    ([("n", "int"), ("y", np.float32, 4)], "stencil", "global i => write y[i]", "INVALID"),   # rank 4
    ([("n", "int"), ("y", np.float32, 1)], "not a name", "global i => write y[i]", "INVALID"),
    ([("n", "int"), ("y", np.float32, 1)], "stencil", "global i => write z[i]", "PARSE"),     # unknown array
    ([("n", "int"), ("y", np.float32, 1)], "stencil", "global i => write y[i*i]", "PARSE"),   # not affine
    ([("n", "int"), ("y", np.float32, 1)], "stencil", "global => write y[0]", "PARSE"),       # binds nothing
])
def test_definition_errors(params, fn, ann, status):
    ctx = dry()
    with pytest.raises(L.LtError) as e:
        ctx.define_source("k", STENCIL, fn, params, ann)
    assert e.value.status == getattr(L, "LT_ERR_" + status)
    ctx.close()


def test_constant_array_parameter_is_rejected():
    ctx = dry()
    with pytest.raises(L.LtError) as e:
        ctx.define_source("k", STENCIL, "stencil", [("n", "int"), ("output", np.float32, 1, "const"),
                                                    ("input", np.float32, 1)], ANN)
    assert e.value.status == L.LT_ERR_INVALID
    ctx.close()


def test_grid_rank_comes_from_the_annotation():
    ctx = dry()
    ctx.define_source("k", STENCIL, "stencil", PARAMS, ANN)
    n = 100
    x = ctx.array([n])
    y = ctx.array([n])
    with pytest.raises(L.LtError) as e:
        ctx.launch("k", [n, 1], [1, 1], [0, 0], args=[n, y, x])
    assert e.value.status == L.LT_ERR_INVALID
    ctx.launch("k", [n], [64], [0], args=[n, y, x])
    ctx.sync()
    ctx.close()


def test_block_over_1024_threads_is_rejected():
    ctx = dry()
    ctx.define_source("k", STENCIL, "stencil", PARAMS, ANN)
    n = 1 << 12
    x = ctx.array([n])
    y = ctx.array([n])
    with pytest.raises(L.LtError) as e:
        ctx.launch("k", [n], [2048], [0], args=[n, y, x])
    assert e.value.status == L.LT_ERR_INVALID
    ctx.close()


def test_user_kernels_do_not_run_in_a_batch():
    ctx = dry()
    ctx.define_source("k", STENCIL, "stencil", PARAMS, ANN)
    n = 1 << 12
    x = ctx.array([n])
    y = ctx.array([n])
    ctx.batch_begin()
    with pytest.raises(L.LtError) as e:
        ctx.launch("k", [n], [64], [1024], args=[n, y, x])
    assert e.value.status == L.LT_ERR_UNSUPPORTED
    ctx.batch_end()
    ctx.close()
