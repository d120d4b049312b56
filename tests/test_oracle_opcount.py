"""Operation count of one oracle step (oracle/opcount.cpp: the oracle's own
source compiled with a floating-point type that counts every operation)."""
import oracle


def test_count_is_the_same_at_every_site():
    # a step does the same arithmetic at every site (periodic grid, no
    # boundaries), so each count is exactly proportional to the sites
    for lat, a, b in ((oracle.D2Q9, 8, 12), (oracle.D3Q19, 4, 6)):
        for mrt in (False, True):
            ca, cb = oracle.opcount(lat, a, mrt), oracle.opcount(lat, b, mrt)
            assert ca["flops_per_site"] == cb["flops_per_site"]
            for k in ("add", "mul", "div", "sqrt"):
                assert ca[k] * cb["sites"] == cb[k] * ca["sites"], (lat, mrt, k)


def test_count_has_no_data_dependent_work():
    # no comparison of floating-point values and no square root in a step:
    # the arithmetic does not depend on the state (S enters only the
    # observables)
    for lat in (oracle.D2Q9, oracle.D3Q19):
        c = oracle.opcount(lat, 4)
        assert c["cmp"] == 0 and c["sqrt"] == 0, c


def test_count_orders():
    d2, d3 = oracle.opcount(oracle.D2Q9, 8), oracle.opcount(oracle.D3Q19, 4)
    assert d3["flops_per_site"] > d2["flops_per_site"]
    # the moment-space collision (two products with the q x q basis) costs
    # more than BGK; the isotropic stencils read every lattice neighbour
    assert oracle.opcount(oracle.D3Q19, 4, mrt=True)["flops_per_site"] > d3["flops_per_site"]
    assert oracle.opcount(oracle.D3Q19, 4, stencil="isotropic")["flops_per_site"] > d3["flops_per_site"]
    assert oracle.opcount(oracle.D2Q9, 8, stencil="isotropic")["flops_per_site"] > d2["flops_per_site"]
    print("oracle flops per site and step: D2Q9 %.0f, D3Q19 %.0f" % (d2["flops_per_site"], d3["flops_per_site"]))
