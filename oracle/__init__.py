"""CPU oracle of the non-equilibrium Renyi-entropy estimator.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in
__graft_entry__.py and the CPU-baseline leg of bench.py may import this
package.  The product package (paper_2304_03311_amd) never imports it and
shares no code with it.
"""
