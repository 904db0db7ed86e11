"""The defaults of the optimizer and of the morphological filters are the
paper's Appendix B values (b1 = 0.9, b2 = 0.999, eta = 0.001, gamma = 0.95,
u0 = 0.01, beta_min = 10, filter sharpness 20), in the product and in the
oracle alike."""
import inspect

from oracle import optimize as oracle_opt

APP_B = dict(b1=0.9, b2=0.999, lr=1e-3, gamma=0.95, u0=0.01, beta_min=10.0)


def defaults(fn):
    return {k: v.default for k, v in inspect.signature(fn).parameters.items()
            if v.default is not inspect.Parameter.empty}


def test_product_optimizer_defaults_are_appendix_b():
    from paper_2505_03352_amd import optimize
    d = defaults(optimize.optimize)
    for k, v in APP_B.items():
        assert d[k] == v, k
    bc = optimize.BetaControl()
    assert (bc.beta_min, bc.gamma, bc.u0) == (10.0, 0.95, 0.01)


def test_oracle_optimizer_defaults_are_appendix_b():
    d = defaults(oracle_opt.optimize)
    for k, v in APP_B.items():
        assert d[k] == v, k
    bc = oracle_opt.BetaControl()
    assert (bc.beta_min, bc.gamma, bc.u0) == (10.0, 0.95, 0.01)
    a = defaults(oracle_opt.adam_step)
    assert (a["lr"], a["b1"], a["b2"]) == (1e-3, 0.9, 0.999)


def test_filter_sharpness_default_is_appendix_b():
    from workloads.devices import Device
    assert Device.__dataclass_fields__["morph_alpha"].default == 20.0
