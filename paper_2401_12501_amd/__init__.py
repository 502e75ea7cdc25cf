"""pmx: parametrix remainder-operator apply and solve for elliptic surface PDEs on MI355X.

Importing the package loads nothing native; ``paper_2401_12501_amd.pmx`` holds
the binding to the HIP library and loads it on first use.
"""
