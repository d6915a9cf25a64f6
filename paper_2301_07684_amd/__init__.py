"""MI355X-native strong-field QED Monte Carlo step (SFQEDtoolkit method, arXiv:2301.07684).

    from paper_2301_07684_amd import sfq      # binding of the C ABI (include/sfq.h)
    h = sfq.Handle(ref_length=..., dt=...)

Submodules: ``sfq`` (binding), ``inputs`` (seeded synthetic workloads), ``tablegen`` (offline
table generator), ``build`` (compiles the HIP library), ``serve`` (continuous-batching server),
``autotune`` (launch-shape tuner).
"""
__all__ = ["sfq", "inputs", "tablegen", "build"]
